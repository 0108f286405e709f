// Sampled counting of order-5 higher-order motifs (Section 6.4 applies the
// sampling algorithm of Section 5 at order 5, where exact counting does not
// reach).
//
// Algorithm 4 at order 5: every sampled hyperedge e of size j (j = 2..5)
// takes every 5-node set V containing e whose induced sub-hypergraph is
// connected and holds no hyperedge larger than e; such a V lies within
// 5 - j hops of e through hyperedges of size at most j.  One workgroup per
// sample lists that ball in LDS (a hash set and a list), then its threads
// stride over the C(|ball|, 5 - j) choices of the other nodes, fill each set
// in (26 subsets: pairs, triples, quadruples and the set itself, Section 4.3)
// and classify it.
//
// At order 5 there are 2^26 patterns, too many for a lookup table in LDS:
// the class of a pattern is computed on the fly as its smallest value over
// the 120 relabellings of the five local positions (ascending node id), and
// classes are reported by that canonical value.  Counts gather in an LDS
// table per workgroup and then in a device hash table; the host sorts the
// classes by canonical value and scales them: est = raw |E_j| / (S_j
// countmax), j the class's largest hyperedge size and countmax the number of
// its hyperedges of that size.
#include <algorithm>
#include <cmath>
#include <vector>

#include "hm_items.h"

namespace hm {

int sample_sizes(const hm_graph* H, int k, double fraction, int allocation, uint64_t* S);

namespace {

constexpr int kSub5 = 26;
constexpr uint32_t kBallCap = 4096;           // ball nodes per sample
constexpr uint32_t kLocalCap = 1024;          // classes cached per workgroup
constexpr uint32_t kThreads5 = 256;
constexpr uint64_t kMaxCandidates = 1ull << 32;   // per sample
constexpr uint32_t kErrBall = 1u, kErrWork = 2u, kErrTable = 4u;

struct Tables5 {
  uint8_t sub_mask[kSub5];       // subset masks of {0..4} with >= 2 members, ascending
  int8_t bit_of_mask[32];
  uint8_t perm[120][5];
};

Tables5 make_tables5() {
  Tables5 t{};
  int n = 0;
  for (int m = 0; m < 32; ++m) {
    t.bit_of_mask[m] = -1;
    if (__builtin_popcount(m) >= 2) {
      t.bit_of_mask[m] = int8_t(n);
      t.sub_mask[n++] = uint8_t(m);
    }
  }
  uint8_t p[5] = {0, 1, 2, 3, 4};
  int q = 0;
  do {
    for (int i = 0; i < 5; ++i) t.perm[q][i] = p[i];
    ++q;
  } while (std::next_permutation(p, p + 5));
  return t;
}

// ------------------------------------------------------------------ 5-node hyperedges
__device__ inline unsigned long long hash5(const uint32_t* m) {
  unsigned long long h = 0x6a09e667f3bcc909ull;
  for (int i = 0; i < 5; ++i) h = mix64(h ^ (m[i] + 0x9e3779b97f4a7c15ull * uint64_t(i + 1)));
  return h;
}

// every unique hyperedge of size 5 of the all-hyperedges list: flags
__global__ void k_e5_flags(const unsigned long long* __restrict__ off, uint64_t n, uint32_t* __restrict__ flag) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
    flag[i] = off[i + 1] - off[i] == 5 ? 1u : 0u;
}

__global__ void k_e5_gather(const unsigned long long* __restrict__ off, const uint32_t* __restrict__ members, uint64_t n,
                            const uint32_t* __restrict__ flag, const uint32_t* __restrict__ pos, uint32_t* __restrict__ e5) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
    if (flag[i])
      for (int j = 0; j < 5; ++j) e5[5ull * pos[i] + j] = members[off[i] + j];
}

__global__ void k_e5_insert(const uint32_t* __restrict__ e5, uint64_t n5, uint32_t* slots, unsigned long long mask) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n5; i += uint64_t(gridDim.x) * blockDim.x) {
    unsigned long long h = hash5(e5 + 5 * i) & mask;
    while (atomicCAS(&slots[h], 0u, uint32_t(i + 1)) != 0u) h = (h + 1) & mask;
  }
}

__device__ inline bool has5(const uint32_t* __restrict__ e5, const uint32_t* __restrict__ slots, unsigned long long mask,
                            const uint32_t* m) {
  if (!slots) return false;
  unsigned long long h = hash5(m) & mask;
  for (;;) {
    const uint32_t s = slots[h];
    if (s == 0u) return false;
    const uint32_t* r = e5 + 5ull * (s - 1);
    if (r[0] == m[0] && r[1] == m[1] && r[2] == m[2] && r[3] == m[3] && r[4] == m[4]) return true;
    h = (h + 1) & mask;
  }
}

// ------------------------------------------------------------------ the counting kernel
struct Sampled5Args {
  View v;
  const uint32_t* e5;
  const uint32_t* hs5;
  unsigned long long hs5_mask;
  const uint32_t* idx[6];       // explicit draws per stratum, or null: drawn here
  uint64_t S[6];                // draws per stratum
  uint64_t n[6];                // |E_j|
  uint64_t seed;
  // device class table: key = canonical + 1 (0 empty), count
  uint32_t* keys;
  unsigned long long* counts;
  unsigned long long mask;
  uint32_t* err;
};

__device__ inline const uint32_t* edge_row(const Sampled5Args& a, int j, uint64_t i) {
  return j == 2 ? a.v.e2 + 2 * i : j == 3 ? a.v.e3 + 3 * i : j == 4 ? a.v.e4 + 4 * i : a.e5 + 5 * i;
}

__device__ inline void add_global(const Sampled5Args& a, uint32_t canon, unsigned long long cnt) {
  const uint32_t key = canon + 1u;
  unsigned long long h = mix64(canon) & a.mask;
  for (uint64_t probes = 0; probes <= a.mask; ++probes) {
    const uint32_t cur = atomicCAS(&a.keys[h], 0u, key);
    if (cur == 0u || cur == key) {
      atomicAdd(&a.counts[h], cnt);
      return;
    }
    h = (h + 1) & a.mask;
  }
  atomicOr(a.err, kErrTable);
}

// fill-in of the 5-node set V (ascending): bit b for the b-th subset
// The subsets of the five local positions with at least two members, in
// ascending mask order (the order of Tables5::sub_mask and of the pattern's
// bits), as constants so that fill5's loops unroll to fixed subsets.
constexpr uint8_t kSubMask5[kSub5] = {3,  5,  6,  7,  9,  10, 11, 12, 13, 14, 15, 17, 18,
                                      19, 20, 21, 22, 23, 24, 25, 26, 27, 28, 29, 30, 31};

// The 26-bit pattern of the ascending 5-node set V: bit b set when subset b
// of V is a hyperedge.  The home slots of the ten 3-node and five 4-node
// subsets are loaded before any probe is resolved, so that their latencies
// overlap; a probe that meets another key continues from there.
__device__ inline uint32_t fill5(const Sampled5Args& a, const Tables5& T, const uint32_t* V) {
  (void)T;
  uint32_t p = 0;
  ulonglong2 home[kSub5];
#pragma unroll
  for (int b = 0; b < kSub5; ++b) {
    const uint32_t m = kSubMask5[b];
    const int n = __builtin_popcount(m);
    uint32_t x[5];
    int k = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i)
      if ((m >> i) & 1u) x[k++] = V[i];
    if (n == 2) {
      p |= pair_bit(a.v.hs2, a.v.bits, a.v.W, x[0], x[1]) << b;
    } else if (n == 3 || n == 4) {
      const Key128 key = n == 3 ? key3(x[0], x[1], x[2]) : key4(x[0], x[1], x[2], x[3]);
      const Set128& set = n == 3 ? a.v.hs3 : a.v.hs4;
      home[b] = *reinterpret_cast<const ulonglong2*>(set.slot + 2 * (hash128(key) & set.mask));
    }
  }
#pragma unroll
  for (int b = 0; b < kSub5; ++b) {
    const uint32_t m = kSubMask5[b];
    const int n = __builtin_popcount(m);
    uint32_t x[5];
    int k = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i)
      if ((m >> i) & 1u) x[k++] = V[i];
    if (n == 3 || n == 4) {
      const Key128 key = n == 3 ? key3(x[0], x[1], x[2]) : key4(x[0], x[1], x[2], x[3]);
      const Set128& set = n == 3 ? a.v.hs3 : a.v.hs4;
      bool has = false;
      ulonglong2 v = home[b];
      if (v.x == key.hi && v.y == key.lo) {
        has = true;
      } else if (v.x != kEmpty64) {
        Probe128 pr;
        pr.key = key;
        pr.pos = ((hash128(key) & set.mask) + 1) & set.mask;
        pr.v = *reinterpret_cast<const ulonglong2*>(set.slot + 2 * pr.pos);
        has = probe128_end(set, pr);
      }
      p |= uint32_t(has) << b;
    } else if (n == 5) {
      p |= uint32_t(has5(a.e5, a.hs5, a.hs5_mask, x)) << b;
    }
  }
  return p;
}

__device__ inline bool connected5(const Tables5& T, uint32_t p) {
  uint32_t adj[5] = {0, 0, 0, 0, 0};
  uint32_t covered = 0;
  for (int b = 0; b < kSub5; ++b)
    if ((p >> b) & 1u) {
      const uint32_t m = T.sub_mask[b];
      covered |= m;
      for (int i = 0; i < 5; ++i)
        if ((m >> i) & 1u) adj[i] |= m;
    }
  if (covered != 31u) return false;
  uint32_t reach = 1u, prev = 0u;
  while (reach != prev) {
    prev = reach;
    for (int i = 0; i < 5; ++i)
      if ((reach >> i) & 1u) reach |= adj[i];
  }
  return reach == 31u;
}

__device__ inline int maxcard5(const Tables5& T, uint32_t p) {
  int mc = 0;
  for (int b = 0; b < kSub5; ++b)
    if ((p >> b) & 1u) mc = max(mc, __popc(T.sub_mask[b]));
  return mc;
}

__device__ inline uint32_t canonical5(const Tables5& T, uint32_t p) {
  uint32_t best = 0xFFFFFFFFu;
  for (int g = 0; g < 120; ++g) {
    uint32_t q = 0;
    for (uint32_t r = p; r; r &= r - 1) {
      const uint32_t m = T.sub_mask[__ffs(r) - 1];
      uint32_t img = 0;
      for (int i = 0; i < 5; ++i)
        if ((m >> i) & 1u) img |= 1u << T.perm[g][i];
      q |= 1u << T.bit_of_mask[img];
    }
    best = min(best, q);
  }
  return best;
}

// largest k with C(k, r) <= t (r = 1, 2, 3), k >= r - 1
__device__ inline uint64_t binom(uint64_t n, int r) {
  return r == 1 ? n : r == 2 ? n * (n - 1) / 2 : n * (n - 1) * (n - 2) / 6;
}

__device__ inline uint64_t colex_top(uint64_t t, int r) {
  double x = r == 1 ? double(t) : r == 2 ? sqrt(2.0 * double(t)) : cbrt(6.0 * double(t));
  uint64_t k = uint64_t(x) + 2;
  while (k > uint64_t(r - 1) && binom(k, r) > t) --k;
  while (binom(k + 1, r) <= t) ++k;
  return k;
}

// LDS of a workgroup
struct Lds5 {
  Tables5 T;
  uint32_t set[2 * kBallCap];     // open addressing, node + 1 (0 empty)
  uint32_t ball[kBallCap];
  uint32_t n_ball;
  uint32_t overflow;
  uint32_t lkeys[kLocalCap];      // (stratum << 26 | raw pattern) + 1 (add_local)
  unsigned long long lcount[kLocalCap];
};

__device__ inline bool ball_insert(Lds5& L, uint32_t node) {
  uint32_t h = uint32_t(mix64(node)) & (2 * kBallCap - 1);
  for (uint32_t probes = 0; probes < 2 * kBallCap; ++probes) {
    const uint32_t cur = atomicCAS(&L.set[h], 0u, node + 1u);
    if (cur == 0u) return true;
    if (cur == node + 1u) return false;
    h = (h + 1) & (2 * kBallCap - 1);
  }
  return false;
}

// The workgroup's counts are kept by raw pattern p and the stratum j of the
// sample (key (j << 26 | p) + 1, 0 empty): patterns repeat across a sample's
// candidate sets, so each distinct one is put in canonical form once, when
// the table is flushed, rather than once per set.  A set that finds no room
// goes to the class table at once.
constexpr uint32_t kPatBits5 = 26;
__device__ inline void add_local(Lds5& L, const Sampled5Args& a, uint32_t j, uint32_t p) {
  const uint32_t key = ((j << kPatBits5) | p) + 1u;
  uint32_t h = uint32_t(mix64(key)) & (kLocalCap - 1);
  for (int probes = 0; probes < 16; ++probes) {
    const uint32_t cur = atomicCAS(&L.lkeys[h], 0u, key);
    if (cur == 0u || cur == key) {
      atomicAdd(&L.lcount[h], 1ull);
      return;
    }
    h = (h + 1) & (kLocalCap - 1);
  }
  add_global(a, canonical5(L.T, p), 1ull);
}

// Sample s of the launch: its stratum j and the position i of its hyperedge
// in that stratum (explicit, or drawn from the seed).
__device__ inline void sample_of(const Sampled5Args& a, uint64_t s, int* j_out, uint64_t* i_out) {
  int j = 2;
  uint64_t r = s;
  while (r >= a.S[j]) r -= a.S[j++];
  *j_out = j;
  *i_out = a.idx[j] ? a.idx[j][r]
                    : bounded64(philox4x64_10(r, 0, 0, 0, a.seed, (kDomainSample << 32) | uint64_t(j)).v[0], a.n[j]);
}

// The ball of a sampled hyperedge e (j nodes): every node within 5 - j hops
// of e through hyperedges of size 2..4 (and, for j = 5, none), e's own
// nodes left out, in L.ball[0 .. L.n_ball) in ascending node order, so that
// every workgroup that builds it enumerates the same candidate sets in the
// same order.  Returns false (L.overflow set) when it holds more than
// kBallCap nodes.  Every thread of the workgroup calls this.
__device__ bool ball5(Lds5& L, const Sampled5Args& a, const uint32_t* e, int j) {
  const int need = 5 - j;
  __syncthreads();   // the previous ball is no longer read
  for (uint32_t x = threadIdx.x; x < 2 * kBallCap; x += blockDim.x) L.set[x] = 0u;
  if (threadIdx.x == 0) {
    L.n_ball = 0;
    L.overflow = 0;
  }
  __syncthreads();
  if (threadIdx.x < uint32_t(j)) ball_insert(L, e[threadIdx.x]);
  __syncthreads();
  // breadth-first: hop h takes the nodes added by hop h - 1 (e itself first)
  uint32_t f0 = 0, f1 = 0;
  for (int h = 0; h < need; ++h) {
    const uint32_t nf = h == 0 ? uint32_t(j) : f1 - f0;
    const int wv = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    for (uint32_t q = wv; q < nf; q += kThreads5 / kWave) {
      const uint32_t u = h == 0 ? e[q] : L.ball[f0 + q];
      // pairs
      for (uint32_t t = a.v.g2_off[u] + lane; t < a.v.g2_off[u + 1]; t += kWave) {
        const uint32_t w = a.v.g2_adj[t];
        if (ball_insert(L, w)) {
          const uint32_t at = atomicAdd(&L.n_ball, 1u);
          if (at < kBallCap) L.ball[at] = w; else L.overflow = 1u;
        }
      }
      for (int fs = 3; fs <= j && fs <= 4; ++fs) {
        const uint32_t* off = fs == 3 ? a.v.i3_off : a.v.i4_off;
        const uint32_t* idx = fs == 3 ? a.v.i3_idx : a.v.i4_idx;
        const uint32_t* rows = fs == 3 ? a.v.e3 : a.v.e4;
        for (uint32_t t = off[u] + lane; t < off[u + 1]; t += kWave) {
          const uint32_t* f = rows + uint64_t(fs) * idx[t];
          for (int m = 0; m < fs; ++m)
            if (ball_insert(L, f[m])) {
              const uint32_t at = atomicAdd(&L.n_ball, 1u);
              if (at < kBallCap) L.ball[at] = f[m]; else L.overflow = 1u;
            }
        }
      }
    }
    __syncthreads();
    f0 = h == 0 ? 0u : f1;
    f1 = min(L.n_ball, kBallCap);
    if (L.overflow) break;
  }
  if (L.overflow) return false;
  // ascending order (bitonic sort in LDS, padded with ~0 to a power of two)
  const uint32_t nb = L.n_ball;
  uint32_t pad = 1;
  while (pad < nb) pad <<= 1;
  for (uint32_t x = nb + threadIdx.x; x < pad; x += blockDim.x) L.ball[x] = 0xFFFFFFFFu;
  __syncthreads();
  for (uint32_t k = 2; k <= pad; k <<= 1)
    for (uint32_t d = k >> 1; d > 0; d >>= 1) {
      for (uint32_t x = threadIdx.x; x < pad; x += blockDim.x) {
        const uint32_t y = x ^ d;
        if (y <= x) continue;
        const uint32_t vx = L.ball[x], vy = L.ball[y];
        if ((vx > vy) == ((x & k) == 0)) {
          L.ball[x] = vy;
          L.ball[y] = vx;
        }
      }
      __syncthreads();
    }
  return true;
}

// Candidate sets of a sample: the choices of 5 - j ball nodes (one set, e
// itself, when j = 5).
__device__ inline uint64_t candidates5(uint32_t nb, int j) {
  const int need = 5 - j;
  return need ? (nb >= uint64_t(need) ? binom(nb, need) : 0) : 1;
}

// Pass 1: every sample's number of candidate chunks (kChunk5 candidate sets
// each; 0 when its ball or its candidates are too many, with the error bit
// set).  One workgroup per sample.
constexpr uint64_t kChunk5 = 1ull << 16;
__global__ void __launch_bounds__(kThreads5) k_chunks5(Sampled5Args a, uint64_t total, uint32_t* __restrict__ chunks) {
  __shared__ Lds5 L;
  for (uint64_t s = blockIdx.x; s < total; s += gridDim.x) {
    int j;
    uint64_t i;
    sample_of(a, s, &j, &i);
    const uint32_t* e = edge_row(a, j, i);
    uint32_t c = 0;
    if (!ball5(L, a, e, j)) {
      if (threadIdx.x == 0) atomicOr(a.err, kErrBall);
    } else {
      const uint64_t cand = candidates5(L.n_ball, j);
      if (cand >= kMaxCandidates) {
        if (threadIdx.x == 0) atomicOr(a.err, kErrWork);
      } else {
        c = uint32_t((cand + kChunk5 - 1) / kChunk5);
      }
    }
    if (threadIdx.x == 0) chunks[s] = c;
  }
}

// Pass 2: the tasks (sample, chunk), tasks [first[s], first[s + 1]) being
// sample s's chunks (first: exclusive scan of the chunk counts, first[total]
// their sum).  A workgroup takes tasks in turn, rebuilds the task's ball and
// classifies the task's candidate sets: with the ball in ascending order,
// candidate t is the t-th choice of 5 - j ball nodes in colex order.
__global__ void __launch_bounds__(kThreads5) k_sampled5(Sampled5Args a, Tables5 tables, uint64_t total,
                                                        const uint32_t* __restrict__ first) {
  __shared__ Lds5 L;
  for (uint32_t i = threadIdx.x; i < kLocalCap; i += blockDim.x) {
    L.lkeys[i] = 0u;
    L.lcount[i] = 0ull;
  }
  if (threadIdx.x == 0) L.T = tables;
  const uint32_t n_tasks = first[total];
  for (uint32_t task = blockIdx.x; task < n_tasks; task += gridDim.x) {
    // the sample whose task range holds `task`
    uint64_t lo = 0, hi = total;   // first[lo] <= task < first[hi]
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) >> 1;
      if (first[mid] <= task) lo = mid; else hi = mid;
    }
    const uint64_t s = lo;
    int j;
    uint64_t i;
    sample_of(a, s, &j, &i);
    const uint32_t* e = edge_row(a, j, i);
    const int need = 5 - j;
    if (!ball5(L, a, e, j)) continue;   // (pass 1 gave it no task)
    const uint64_t cand = candidates5(L.n_ball, j);
    const uint64_t c0 = uint64_t(task - first[s]) * kChunk5, c1 = min(cand, c0 + kChunk5);
    for (uint64_t t = c0 + threadIdx.x; t < c1; t += blockDim.x) {
      uint32_t V[5];
      for (int m = 0; m < j; ++m) V[m] = e[m];
      // the t-th choice of `need` ball nodes, colex order
      uint64_t rest = t;
      for (int rr = need; rr >= 1; --rr) {
        const uint64_t top = colex_top(rest, rr);
        rest -= binom(top, rr);
        V[j + need - rr] = L.ball[top];
      }
      for (int x = 1; x < 5; ++x) {   // ascending node ids
        const uint32_t y = V[x];
        int z = x - 1;
        while (z >= 0 && V[z] > y) {
          V[z + 1] = V[z];
          --z;
        }
        V[z + 1] = y;
      }
      const uint32_t p = fill5(a, L.T, V);
      if (maxcard5(L.T, p) != j || !connected5(L.T, p)) continue;
      add_local(L, a, uint32_t(j), p);
    }
  }
  __syncthreads();
  for (uint32_t x = threadIdx.x; x < kLocalCap; x += blockDim.x)
    if (L.lkeys[x])
      add_global(a, canonical5(L.T, (L.lkeys[x] - 1u) & ((1u << kPatBits5) - 1u)), L.lcount[x]);
}

// compact the device class table: flags then positions
__global__ void k_class_flags(const uint32_t* __restrict__ keys, uint64_t n, uint32_t* __restrict__ flag) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
    flag[i] = keys[i] ? 1u : 0u;
}

__global__ void k_class_compact(const uint32_t* __restrict__ keys, const unsigned long long* __restrict__ counts,
                                uint64_t n, const uint32_t* __restrict__ flag, const uint32_t* __restrict__ pos,
                                unsigned long long* __restrict__ sort_keys, uint32_t* __restrict__ sort_vals,
                                unsigned long long* __restrict__ cnt_out) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
    if (flag[i]) {
      sort_keys[pos[i]] = keys[i] - 1u;
      sort_vals[pos[i]] = pos[i];
      cnt_out[pos[i]] = counts[i];
    }
}

struct Scale5 {
  double n[6];
  double s[6];
};

// classes in canonical order: canonical, raw count, estimate (Algorithm 4's
// correction, fp64 rounded once to fp32)
__global__ void k_finish5(const unsigned long long* __restrict__ sorted_canon, const uint32_t* __restrict__ order,
                          const unsigned long long* __restrict__ cnt, uint64_t n, Scale5 sc, Tables5 T,
                          uint32_t* __restrict__ canon_out, int64_t* __restrict__ raw_out, float* __restrict__ est_out) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x) {
    const uint32_t c = uint32_t(sorted_canon[i]);
    const unsigned long long r = cnt[order[i]];
    int mc = 0, cm = 0;
    for (int b = 0; b < kSub5; ++b)
      if ((c >> b) & 1u) {
        const int sz = __popc(T.sub_mask[b]);
        if (sz > mc) {
          mc = sz;
          cm = 1;
        } else if (sz == mc) {
          ++cm;
        }
      }
    canon_out[i] = c;
    raw_out[i] = int64_t(r);
    est_out[i] = sc.s[mc] > 0.0 ? float(double(r) * sc.n[mc] / (sc.s[mc] * double(cm))) : 0.f;
  }
}

unsigned grid5(uint64_t n) {
  uint64_t g = (n + 255) / 256;
  return unsigned(std::max<uint64_t>(1, std::min<uint64_t>(g, 4096)));
}

}  // namespace

// E_5 and its hash set, on first use.
int ensure_order5(hm_graph* H, hipStream_t st) {
  if (H->order5_built) return HM_OK;
  note_use(H, st);
  const uint64_t n = H->n_unique;
  std::vector<void*> tmp;
  struct Free {
    std::vector<void*>& t;
    hipStream_t st;
    ~Free() { dfree_on(t.data(), t.size(), st); }
  } release{tmp, st};
  auto get = [&](void** p, size_t bytes) {
    int rc = dalloc(p, bytes ? bytes : 4);
    if (rc == HM_OK) tmp.push_back(*p);
    return rc;
  };
  void *flag = nullptr, *pos = nullptr, *tot = nullptr;
  HM_TRY(get(&flag, (n + 1) * 4));
  HM_TRY(get(&pos, (n + 1) * 4));
  HM_TRY(get(&tot, 8));
  uint32_t n5 = 0;
  if (n) {
    k_e5_flags<<<grid5(n), 256, 0, st>>>(H->all_off, n, static_cast<uint32_t*>(flag));
    HM_HIP(hipGetLastError());
    HM_TRY(scan_exclusive_u32(static_cast<uint32_t*>(flag), static_cast<uint32_t*>(pos), n,
                              static_cast<uint32_t*>(tot), st));
    HM_HIP(hipMemcpyAsync(&n5, tot, 4, hipMemcpyDeviceToHost, st));
    HM_HIP(hipStreamSynchronize(st));
  }
  void *e5 = nullptr, *slots = nullptr;
  const unsigned long long cap = pow2_capacity(n5);
  HM_TRY(dalloc(&e5, size_t(n5 ? n5 : 1) * 5 * 4));
  int rc = dalloc(&slots, size_t(cap) * 4);
  if (rc != HM_OK) {
    dfree(e5);
    return rc;
  }
  rc = fill_u32(static_cast<uint32_t*>(slots), 0u, cap, st);
  if (rc == HM_OK && n5) {
    k_e5_gather<<<grid5(n), 256, 0, st>>>(H->all_off, H->all_members, n, static_cast<uint32_t*>(flag),
                                          static_cast<uint32_t*>(pos), static_cast<uint32_t*>(e5));
    k_e5_insert<<<grid5(n5), 256, 0, st>>>(static_cast<uint32_t*>(e5), n5, static_cast<uint32_t*>(slots), cap - 1);
    if (hipGetLastError() != hipSuccess) rc = HM_EDEVICE;
  }
  if (rc == HM_OK && hipStreamSynchronize(st) != hipSuccess) rc = HM_EDEVICE;
  if (rc != HM_OK) {
    dfree(e5);
    dfree(slots);
    return rc;
  }
  H->e5 = static_cast<uint32_t*>(e5);
  H->hs5 = static_cast<uint32_t*>(slots);
  H->hs5_mask = cap - 1;
  H->n5 = n5;
  H->order5_built = true;
  return HM_OK;
}

// Algorithm 4 at order 5 for the draws S[j] (idx[j] explicit, or drawn from
// seed); synchronous.
int sampled5(hm_graph* H, const uint32_t* const idx[6], const uint64_t S[6], uint64_t seed, uint64_t capacity,
             uint32_t* canon, int64_t* raw, float* est, uint64_t* n_classes, hipStream_t st) {
  HM_TRY(ensure_order5(H, st));
  note_use(H, st);
  Sampled5Args a{};
  a.v = view_of(H);
  a.e5 = H->e5;
  a.hs5 = H->n5 ? H->hs5 : nullptr;
  a.hs5_mask = H->hs5_mask;
  const uint64_t nj[6] = {0, 0, H->n_by_size[2], H->n_by_size[3], H->n_by_size[4], H->n5};
  uint64_t total = 0;
  for (int j = 0; j < 6; ++j) {
    a.idx[j] = j >= 2 ? idx[j] : nullptr;
    a.n[j] = nj[j];
    a.S[j] = (j >= 2 && nj[j]) ? S[j] : 0;
    total += a.S[j];
  }
  a.seed = seed;
  // the device class table: at most one class per candidate set, bounded by
  // the 2^26 patterns; sized for the output capacity at load 1/2
  const unsigned long long tcap = pow2_capacity(std::min<uint64_t>(std::max<uint64_t>(capacity, 1024), 1ull << 26));
  std::vector<void*> tmp;
  struct Free {
    std::vector<void*>& t;
    hipStream_t st;
    ~Free() { dfree_on(t.data(), t.size(), st); }
  } release{tmp, st};
  auto get = [&](void** p, size_t bytes) {
    int rc = dalloc(p, bytes ? bytes : 8);
    if (rc == HM_OK) tmp.push_back(*p);
    return rc;
  };
  void *keys = nullptr, *counts = nullptr, *err = nullptr;
  HM_TRY(get(&keys, tcap * 4));
  HM_TRY(get(&counts, tcap * 8));
  HM_TRY(get(&err, 8));
  HM_TRY(fill_u32(static_cast<uint32_t*>(keys), 0u, tcap, st));
  HM_TRY(fill_u64(static_cast<unsigned long long*>(counts), 0ull, tcap, st));
  HM_TRY(fill_u32(static_cast<uint32_t*>(err), 0u, 1, st));
  a.keys = static_cast<uint32_t*>(keys);
  a.counts = static_cast<unsigned long long*>(counts);
  a.mask = tcap - 1;
  a.err = static_cast<uint32_t*>(err);
  const Tables5 T = make_tables5();
  if (total) {
    // pass 1: candidate chunks per sample; pass 2: the (sample, chunk) tasks
    void *chunks = nullptr, *first = nullptr;
    HM_TRY(get(&chunks, total * 4));
    HM_TRY(get(&first, (total + 1) * 4));
    k_chunks5<<<unsigned(std::min<uint64_t>(total, 4096)), kThreads5, 0, st>>>(a, total,
                                                                               static_cast<uint32_t*>(chunks));
    HM_HIP(hipGetLastError());
    HM_TRY(scan_exclusive_u32(static_cast<uint32_t*>(chunks), static_cast<uint32_t*>(first), total,
                              static_cast<uint32_t*>(first) + total, st));
    ProfileScope ps("k_sampled5", st);
    k_sampled5<<<4096, kThreads5, 0, st>>>(a, T, total, static_cast<const uint32_t*>(first));
    HM_HIP(hipGetLastError());
  }
  uint32_t host_err = 0;
  HM_HIP(hipMemcpyAsync(&host_err, err, 4, hipMemcpyDeviceToHost, st));
  // compact, sort by canonical value, scale
  void *flag = nullptr, *pos = nullptr, *tot = nullptr;
  HM_TRY(get(&flag, tcap * 4));
  HM_TRY(get(&pos, tcap * 4));
  HM_TRY(get(&tot, 8));
  k_class_flags<<<grid5(tcap), 256, 0, st>>>(a.keys, tcap, static_cast<uint32_t*>(flag));
  HM_HIP(hipGetLastError());
  HM_TRY(scan_exclusive_u32(static_cast<uint32_t*>(flag), static_cast<uint32_t*>(pos), tcap,
                            static_cast<uint32_t*>(tot), st));
  uint32_t nc = 0;
  HM_HIP(hipMemcpyAsync(&nc, tot, 4, hipMemcpyDeviceToHost, st));
  HM_HIP(hipStreamSynchronize(st));
  if (host_err & kErrBall) {
    set_error("order 5: a sampled hyperedge has more than %u nodes within reach", kBallCap);
    return HM_EUNSUPPORTED;
  }
  if (host_err & kErrWork) {
    set_error("order 5: a sampled hyperedge has 2^32 or more candidate node sets");
    return HM_EUNSUPPORTED;
  }
  if (host_err & kErrTable) {
    set_error("order 5: more classes than the class table holds (raise the capacity)");
    return HM_EINVAL;
  }
  *n_classes = nc;
  if (nc > capacity) {
    set_error("order 5: %u classes found, the output holds %llu", nc, (unsigned long long)capacity);
    return HM_EINVAL;
  }
  if (!nc) return HM_OK;
  void *sk = nullptr, *sv = nullptr, *skt = nullptr, *svt = nullptr, *cnt = nullptr;
  HM_TRY(get(&sk, size_t(nc) * 8));
  HM_TRY(get(&sv, size_t(nc) * 4));
  HM_TRY(get(&skt, size_t(nc) * 8));
  HM_TRY(get(&svt, size_t(nc) * 4));
  HM_TRY(get(&cnt, size_t(nc) * 8));
  k_class_compact<<<grid5(tcap), 256, 0, st>>>(a.keys, a.counts, tcap, static_cast<uint32_t*>(flag),
                                               static_cast<uint32_t*>(pos), static_cast<unsigned long long*>(sk),
                                               static_cast<uint32_t*>(sv), static_cast<unsigned long long*>(cnt));
  HM_HIP(hipGetLastError());
  HM_TRY(radix_sort_pairs(static_cast<unsigned long long*>(sk), static_cast<uint32_t*>(sv),
                          static_cast<unsigned long long*>(skt), static_cast<uint32_t*>(svt), nc, 26, st));
  Scale5 sc{};
  for (int j = 2; j <= 5; ++j) {
    sc.n[j] = double(nj[j]);
    sc.s[j] = double(a.S[j]);
  }
  k_finish5<<<grid5(nc), 256, 0, st>>>(static_cast<unsigned long long*>(sk), static_cast<uint32_t*>(sv),
                                       static_cast<unsigned long long*>(cnt), nc, sc, T, canon, raw, est);
  HM_HIP(hipGetLastError());
  HM_HIP(hipStreamSynchronize(st));
  return HM_OK;
}

}  // namespace hm

extern "C" {

int hm_order5_sizes(const hm_graph* H, uint64_t* n_by_size4, void* stream) {
  try {
    if (!H || !n_by_size4) {
      hm::set_error("NULL argument to hm_order5_sizes");
      return HM_EINVAL;
    }
    HM_TRY(hm::ensure_order5(const_cast<hm_graph*>(H), static_cast<hipStream_t>(stream)));
    n_by_size4[0] = H->n_by_size[2];
    n_by_size4[1] = H->n_by_size[3];
    n_by_size4[2] = H->n_by_size[4];
    n_by_size4[3] = H->n5;
    return HM_OK;
  } catch (...) {
    return hm::api_failure();
  }
}

int count_sampled5(const hm_graph* H, double fraction, uint64_t seed, uint64_t capacity, uint32_t* canon, int64_t* raw,
                   float* est, uint64_t* n_classes, void* stream) {
  try {
    if (!H || !canon || !raw || !est || !n_classes) {
      hm::set_error("NULL argument to count_sampled5");
      return HM_EINVAL;
    }
    if (!(fraction > 0.0 && fraction <= 1.0)) {
      hm::set_error("fraction must be in (0, 1]");
      return HM_EINVAL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    HM_TRY(hm::ensure_order5(const_cast<hm_graph*>(H), st));
    const uint64_t nj[6] = {0, 0, H->n_by_size[2], H->n_by_size[3], H->n_by_size[4], H->n5};
    uint64_t S[6] = {0, 0, 0, 0, 0, 0};
    for (int j = 2; j <= 5; ++j) S[j] = uint64_t(std::ceil(fraction * double(nj[j])));
    const uint32_t* idx[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    return hm::sampled5(const_cast<hm_graph*>(H), idx, S, seed, capacity, canon, raw, est, n_classes, st);
  } catch (...) {
    return hm::api_failure();
  }
}

int count_sampled5_indices(const hm_graph* H, const uint32_t* idx2, uint64_t s2, const uint32_t* idx3, uint64_t s3,
                           const uint32_t* idx4, uint64_t s4, const uint32_t* idx5, uint64_t s5, uint64_t capacity,
                           uint32_t* canon, int64_t* raw, float* est, uint64_t* n_classes, void* stream) {
  try {
    if (!H || !canon || !raw || !est || !n_classes) {
      hm::set_error("NULL argument to count_sampled5_indices");
      return HM_EINVAL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    HM_TRY(hm::ensure_order5(const_cast<hm_graph*>(H), st));
    const uint32_t* idx[6] = {nullptr, nullptr, idx2, idx3, idx4, idx5};
    const uint64_t S[6] = {0, 0, s2, s3, s4, s5};
    const uint64_t nj[6] = {0, 0, H->n_by_size[2], H->n_by_size[3], H->n_by_size[4], H->n5};
    for (int j = 2; j <= 5; ++j)
      if (S[j] && (!idx[j] || !nj[j])) {
        hm::set_error("stratum %d: draws without an index array or from an empty stratum", j);
        return HM_EINVAL;
      }
    // every index must lie in its stratum (checked on the host copy)
    for (int j = 2; j <= 5; ++j) {
      if (!S[j]) continue;
      std::vector<uint32_t> h(S[j]);
      HM_HIP(hipMemcpy(h.data(), idx[j], S[j] * 4, hipMemcpyDeviceToHost));
      for (uint32_t x : h)
        if (x >= nj[j]) {
          hm::set_error("a sample index lies outside its stratum");
          return HM_EINVAL;
        }
    }
    return hm::sampled5(const_cast<hm_graph*>(H), idx, S, 0, capacity, canon, raw, est, n_classes, st);
  } catch (...) {
    return hm::api_failure();
  }
}

}  // extern "C"
