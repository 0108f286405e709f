// Randomised null hypergraphs and motif over/under-expression (Section 1 and
// Section 3: motifs are patterns whose frequency differs from that in
// randomised hypergraphs; Section 6.3 draws them from a configuration model).
//
// Null model: stub matching that keeps every node degree and every hyperedge
// size.  The stubs are the members (ascending) of the unique hyperedges of
// size >= 2 in first-occurrence order.  Copy c uses the Philox4x64-10 stream
// key (seed, 2<<32 | c):
//   round 0  order the stubs by (word0 of counter (t, 0, 0, 0), t) and cut the
//            ordered stubs into the original size sequence;
//   round r  (while some hyperedge repeats a node, r = 1..64) the offending
//            hyperedges B (ascending) each get a partner hi64(word0 of counter
//            (q, r, 1, 0) * E); the members of B u partners (ascending
//            hyperedge order, stored member order) are reordered by
//            (word0 of counter (t, r, 0, 0), t) and dealt back in that order.
// Each copy is then counted exactly and z_m = (x_m - mean_m) / sd_m over the
// copies (sd with n - 1) is formed in fp64 and rounded to fp32.
//
// Configuration model (Section 6.3's null; Chodrow, J. Complex Networks 2020):
// Markov chain Monte Carlo with pairwise reshuffles, which keep degrees and
// sizes and whose symmetric moves keep the uniform distribution.  Copy c
// starts from the input's hyperedges and runs `sweeps` rounds with the key
// (seed, 5<<32 | c):
//   round r  order the hyperedges by (word0 of counter (i, r, 0, 0), i) into
//            pi; pair t = (pi[2t], pi[2t+1]); an odd last hyperedge waits;
//   pair t   I = e & f; D = (e - f ascending) then (f - e ascending);
//            a = |e - f|; for q < a: j = q + hi64(w (|D| - q)), w = word
//            (q mod 4) of counter (t, r, 1 + q div 4, 0); swap D[q], D[j];
//            e = sort(I + D[:a]), f = sort(I + D[a:]).
// The motif profile is the relative abundance (x - mu) / (x + mu + eps) of the
// cited higher-order motif work, with its significance profile.
#include <vector>

#include <map>
#include <mutex>
#include <tuple>

#include "hm_items.h"

namespace hm {

int count_exact_impl(const hm_graph* H, int k, int64_t* counts, hipStream_t st);
IdShapes id_shapes(bool on);
int sampled_with_sizes(const hm_graph* H, int k, const uint64_t S[5], uint64_t seed, float* est, int64_t* raw,
                       hipStream_t st);

namespace {

constexpr int kMaxRepairRounds = 64;

// Sorting R copies' random orders at once: item i = c * per + x of copy c
// carries the word w = word 0 of Philox at counter (x, round, 0, 0) under
// key (seed, domain << 32 | c0 + c), and each copy's items are wanted in the
// order of (w, x).  The sort key is (c << 32) | (w >> 32); k_fix_ties then
// orders the rare runs of equal keys by (low half of w, i), which gives the
// order of the full word with ties by position.
__device__ inline unsigned long long order_word(uint64_t i, uint64_t per, uint64_t round, uint32_t c0,
                                                unsigned long long domain, unsigned long long seed) {
  return philox4x64_10(i % per, round, 0, 0, seed, (domain << 32) | (c0 + i / per)).v[0];
}

__global__ void k_order_keys(uint32_t c0, uint32_t R, uint64_t per, uint64_t round, unsigned long long domain,
                             const unsigned long long* __restrict__ seed_p, unsigned long long* keys, uint32_t* vals) {
  const unsigned long long seed = *seed_p;
  const uint64_t n = uint64_t(R) * per;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x) {
    const unsigned long long w = order_word(i, per, round, c0, domain, seed);
    keys[i] = ((unsigned long long)(i / per) << 32) | (w >> 32);
    vals[i] = uint32_t(i);
  }
}

__global__ void k_fix_ties(const unsigned long long* __restrict__ keys, uint32_t* __restrict__ vals, uint64_t n,
                           uint64_t per, uint64_t round, uint32_t c0, unsigned long long domain,
                           const unsigned long long* __restrict__ seed_p) {
  const unsigned long long seed = *seed_p;
  for (uint64_t p = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; p + 1 < n; p += uint64_t(gridDim.x) * blockDim.x) {
    const unsigned long long k = keys[p];
    if (keys[p + 1] != k || (p > 0 && keys[p - 1] == k)) continue;   // not the start of a run
    uint64_t e = p + 2;
    while (e < n && keys[e] == k) ++e;
    // insertion sort of vals[p, e) by (low half of the word, value)
    for (uint64_t i = p + 1; i < e; ++i) {
      const uint32_t v = vals[i];
      const uint32_t lo = uint32_t(order_word(v, per, round, c0, domain, seed));
      uint64_t j = i;
      while (j > p) {
        const uint32_t u = vals[j - 1];
        const uint32_t ulo = uint32_t(order_word(u, per, round, c0, domain, seed));
        if (ulo < lo || (ulo == lo && u < v)) break;
        vals[j] = u;
        --j;
      }
      vals[j] = v;
    }
  }
}

__global__ void k_null_gather(const uint32_t* __restrict__ vals, uint64_t n, uint64_t T,
                              const uint32_t* __restrict__ stubs, uint32_t* __restrict__ members) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x) {
    const uint64_t c = i / T;
    members[i] = stubs[vals[i] - c * T];
  }
}

// ---------------------------------------------------------------- configuration model
constexpr unsigned long long kDomainConfig = 5ull;

// members of every copy := the input's (R x T)
__global__ void k_cfg_init(uint32_t R, uint64_t T, const uint32_t* __restrict__ src, uint32_t* __restrict__ members) {
  const uint64_t n = uint64_t(R) * T;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
    members[i] = src[i % T];
}

// One thread per (copy, pair): the pairwise reshuffle of the two hyperedges
// the sorted order pairs.  members holds copy c's hyperedges at c * T +
// off[e]; tmp (R x T) gives each pair the slots of its two hyperedges as
// working space: virtual slot q < |e| is tmp[c*T + off[e] + q], the rest
// tmp[c*T + off[f] + q - |e|].  D takes slots [0, |D|), I the last |I|.
__global__ void k_cfg_pairs(uint32_t c0, uint32_t R, uint32_t E, uint64_t T, uint32_t r,
                            const unsigned long long* __restrict__ seed_p, const uint32_t* __restrict__ order,
                            const unsigned long long* __restrict__ off, uint32_t* __restrict__ members,
                            uint32_t* __restrict__ tmp) {
  const unsigned long long seed = *seed_p;
  const uint32_t P = E / 2;
  const uint64_t n = uint64_t(R) * P;
  for (uint64_t it = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < n; it += uint64_t(gridDim.x) * blockDim.x) {
    const uint32_t c = uint32_t(it / P), t = uint32_t(it % P);
    const uint64_t base = uint64_t(c) * T;
    const uint32_t ie = order[uint64_t(c) * E + 2 * t] - c * E, jf = order[uint64_t(c) * E + 2 * t + 1] - c * E;
    const uint64_t oe = off[ie], of = off[jf];
    const uint32_t se = uint32_t(off[ie + 1] - oe), sf = uint32_t(off[jf + 1] - of);
    uint32_t* me = members + base + oe;
    uint32_t* mf = members + base + of;
    uint32_t* te = tmp + base + oe;
    uint32_t* tf = tmp + base + of;
    auto slot = [&](uint32_t q) -> uint32_t& { return q < se ? te[q] : tf[q - se]; };
    // two merges of the ascending lists: e - f into D and e & f into I, then
    // f - e after e - f
    uint32_t nd = 0, ni = 0;
    const uint32_t total = se + sf;
    for (uint32_t x = 0, y = 0; x < se;) {
      if (y == sf || me[x] < mf[y]) {
        slot(nd++) = me[x++];
      } else if (mf[y] < me[x]) {
        ++y;
      } else {
        slot(total - 1 - ni++) = me[x];
        ++x;
        ++y;
      }
    }
    const uint32_t a = nd;   // |e - f|
    for (uint32_t x = 0, y = 0; y < sf;) {
      if (x == se || mf[y] < me[x]) {
        slot(nd++) = mf[y++];
      } else if (me[x] < mf[y]) {
        ++x;
      } else {
        ++x;
        ++y;
      }
    }
    Philox4 w{{0, 0, 0, 0}};
    for (uint32_t q = 0; q < a; ++q) {
      if ((q & 3) == 0) w = philox4x64_10(t, r, 1 + q / 4, 0, seed, (kDomainConfig << 32) | (c0 + c));
      const uint32_t j = q + uint32_t(bounded64(w.v[q & 3], nd - q));
      const uint32_t tq = slot(q);
      slot(q) = slot(j);
      slot(j) = tq;
    }
    // e = sort(I + D[:a]), f = sort(I + D[a:]) (insertion sorts into place)
    auto place = [&](uint32_t* out, uint32_t lo, uint32_t hi) {
      uint32_t m = 0;
      for (uint32_t u = 0; u < ni; ++u) {
        const uint32_t v = slot(total - 1 - u);
        uint32_t k = m++;
        while (k > 0 && out[k - 1] > v) {
          out[k] = out[k - 1];
          --k;
        }
        out[k] = v;
      }
      for (uint32_t q = lo; q < hi; ++q) {
        const uint32_t v = slot(q);
        uint32_t k = m++;
        while (k > 0 && out[k - 1] > v) {
          out[k] = out[k - 1];
          --k;
        }
        out[k] = v;
      }
    };
    place(me, 0, a);
    place(mf, a, nd);
  }
}

// delta_m = (x_m - mu_m) / (x_m + mu_m + eps) over R null rows, and the
// significance profile delta / ||delta||_2 (one workgroup, fp64)
__global__ void k_motif_profile(const double* __restrict__ real, const double* __restrict__ nulls, uint32_t R, int C,
                                double eps, double* __restrict__ delta, double* __restrict__ sp) {
  __shared__ double red[256];
  double own = 0.0, sq = 0.0;
  for (int c = threadIdx.x; c < C; c += blockDim.x) {
    double s = 0.0;
    for (uint32_t i = 0; i < R; ++i) s += nulls[uint64_t(i) * C + c];
    const double mu = s / double(R), x = real[c];
    own = (x - mu) / (x + mu + eps);
    if (delta) delta[c] = own;
    sq += own * own;
  }
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (int(threadIdx.x) < d) red[threadIdx.x] += red[threadIdx.x + d];
    __syncthreads();
  }
  const double norm = sqrt(red[0]);
  if (sp)
    for (int c = threadIdx.x; c < C; c += blockDim.x) {
      double s = 0.0;
      for (uint32_t i = 0; i < R; ++i) s += nulls[uint64_t(i) * C + c];
      const double mu = s / double(R), x = real[c];
      const double d = (x - mu) / (x + mu + eps);
      sp[c] = norm > 0.0 ? d / norm : 0.0;
    }
}

__global__ void k_f32_to_f64(const float* __restrict__ a, int n, double* __restrict__ b) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) b[i] = double(a[i]);
}

// Pearson's rho, the largest and the mean absolute error between two
// profiles of C values (one workgroup of 256, fp64, fixed summation order)
__global__ void k_profile_quality(const double* __restrict__ a, const double* __restrict__ b, int C,
                                  double* __restrict__ out) {
  __shared__ double r0[256], r1[256], r2[256];
  double sa = 0.0, sb = 0.0;
  for (int c = threadIdx.x; c < C; c += blockDim.x) {
    sa += a[c];
    sb += b[c];
  }
  r0[threadIdx.x] = sa;
  r1[threadIdx.x] = sb;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (int(threadIdx.x) < d) {
      r0[threadIdx.x] += r0[threadIdx.x + d];
      r1[threadIdx.x] += r1[threadIdx.x + d];
    }
    __syncthreads();
  }
  const double ma = r0[0] / double(C), mb = r1[0] / double(C);
  __syncthreads();
  double sab = 0.0, saa = 0.0, sbb = 0.0, mx = 0.0, sabs = 0.0;
  for (int c = threadIdx.x; c < C; c += blockDim.x) {
    const double da = a[c] - ma, db = b[c] - mb;
    sab += da * db;
    saa += da * da;
    sbb += db * db;
    const double e = fabs(a[c] - b[c]);
    mx = fmax(mx, e);
    sabs += e;
  }
  r0[threadIdx.x] = sab;
  r1[threadIdx.x] = saa;
  r2[threadIdx.x] = sbb;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (int(threadIdx.x) < d) {
      r0[threadIdx.x] += r0[threadIdx.x + d];
      r1[threadIdx.x] += r1[threadIdx.x + d];
      r2[threadIdx.x] += r2[threadIdx.x + d];
    }
    __syncthreads();
  }
  const double s_ab = r0[0], s_aa = r1[0], s_bb = r2[0];
  __syncthreads();
  r0[threadIdx.x] = mx;
  r1[threadIdx.x] = sabs;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (int(threadIdx.x) < d) {
      r0[threadIdx.x] = fmax(r0[threadIdx.x], r0[threadIdx.x + d]);
      r1[threadIdx.x] += r1[threadIdx.x + d];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double den = sqrt(s_aa * s_bb);
    out[0] = den > 0.0 ? s_ab / den : 0.0;
    out[1] = r0[0];
    out[2] = r1[0] / double(C);
  }
}

// ---------------------------------------------------------------- block helpers
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* wsum, uint32_t* total) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const uint32_t x = wave_inclusive_scan(v);
  if (lane == kWave - 1) wsum[wave] = x;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int w = 0; w < kWavesPerBlock; ++w) {
    if (w < wave) before += wsum[w];
    all += wsum[w];
  }
  __syncthreads();
  *total = all;
  return before + x - v;
}

// Stable compaction of the indices i < n with flag(i) into out (ascending).
// Each thread takes kCompactRun consecutive indices per round, so that one
// workgroup scan serves kThreads * kCompactRun of them.
constexpr uint32_t kCompactRun = 4;
template <typename F>
__device__ uint32_t block_compact(uint32_t n, F flag, uint32_t* out, uint32_t* wsum) {
  uint32_t count = 0;
  for (uint32_t base = 0; base < n; base += kThreads * kCompactRun) {
    const uint32_t i0 = base + threadIdx.x * kCompactRun;
    uint32_t bits = 0;
#pragma unroll
    for (uint32_t k = 0; k < kCompactRun; ++k)
      if (i0 + k < n && flag(i0 + k)) bits |= 1u << k;
    uint32_t tot;
    uint32_t pos = block_exclusive_scan(uint32_t(__popc(bits)), wsum, &tot);
#pragma unroll
    for (uint32_t k = 0; k < kCompactRun; ++k)
      if (bits & (1u << k)) out[count + pos++] = i0 + k;
    count += tot;
  }
  __syncthreads();
  return count;
}

// Ascending bitonic sort of n_pad (a power of two) (key, aux) pairs in
// device memory by one workgroup; ties are broken by aux.  Up to
// kLdsBitonic entries the sort runs on copies in LDS (lk, la, lv).
constexpr uint32_t kLdsBitonic = 2048;
__device__ void block_bitonic(unsigned long long* key, uint32_t* aux, uint32_t* val, uint32_t n_pad,
                              unsigned long long* lk, uint32_t* la, uint32_t* lv) {
  if (n_pad <= kLdsBitonic) {
    for (uint32_t i = threadIdx.x; i < n_pad; i += kThreads) {
      lk[i] = key[i];
      la[i] = aux[i];
      if (val) lv[i] = val[i];
    }
    __syncthreads();
    for (uint32_t k = 2; k <= n_pad; k <<= 1)
      for (uint32_t j = k >> 1; j > 0; j >>= 1) {
        for (uint32_t i = threadIdx.x; i < n_pad; i += kThreads) {
          const uint32_t l = i ^ j;
          if (l <= i) continue;
          const bool asc = (i & k) == 0;
          const bool greater = lk[i] > lk[l] || (lk[i] == lk[l] && la[i] > la[l]);
          if (greater == asc) {
            const unsigned long long tk = lk[i];
            lk[i] = lk[l];
            lk[l] = tk;
            const uint32_t ta = la[i];
            la[i] = la[l];
            la[l] = ta;
            if (val) {
              const uint32_t tv = lv[i];
              lv[i] = lv[l];
              lv[l] = tv;
            }
          }
        }
        __syncthreads();
      }
    for (uint32_t i = threadIdx.x; i < n_pad; i += kThreads) {
      key[i] = lk[i];
      aux[i] = la[i];
      if (val) val[i] = lv[i];
    }
    __syncthreads();
    return;
  }
  for (uint32_t k = 2; k <= n_pad; k <<= 1)
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < n_pad; i += kThreads) {
        const uint32_t l = i ^ j;
        if (l <= i) continue;
        const bool asc = (i & k) == 0;
        const bool greater = key[i] > key[l] || (key[i] == key[l] && aux[i] > aux[l]);
        if (greater == asc) {
          const unsigned long long tk = key[i];
          key[i] = key[l];
          key[l] = tk;
          const uint32_t ta = aux[i];
          aux[i] = aux[l];
          aux[l] = ta;
          if (val) {
            const uint32_t tv = val[i];
            val[i] = val[l];
            val[l] = tv;
          }
        }
      }
      __syncthreads();
    }
}

__device__ inline bool repeats_node(const uint32_t* m, uint32_t s) {
  for (uint32_t a = 1; a < s; ++a)
    for (uint32_t b = 0; b < a; ++b)
      if (m[a] == m[b]) return true;
  return false;
}

// Round 1's bad hyperedges of a copy are found by k_null_deal in kBadLists
// lists (hyperedge i in list i % kBadLists, of at most bad_cap entries), each
// with its own counter kBadStride words from the next, so that few
// device-scope atomics meet on one address.
constexpr uint32_t kBadLists = 32;
constexpr uint32_t kBadStride = 32;
struct RepairScratch {
  uint32_t* bad;                 // bad_stride per repair workgroup
  uint32_t* counts;              // per copy: kBadLists counters, kBadStride words apart
  uint32_t bad_cap;              // ceil(E / kBadLists)
  uint64_t bad_stride;           // kBadLists * bad_cap (>= E)
  uint32_t* chosen;              // 2E padded to a power of two
  unsigned long long* key;       // pool keys, padded
  uint32_t* aux;                 // pool positions
  uint32_t* val;                 // pool nodes
  uint32_t* off;                 // pool offsets per chosen hyperedge
  uint64_t chosen_pad;           // capacity of chosen (power of two)
  uint64_t pool_pad;             // capacity of the pool arrays (power of two)
};

// The stub matching dealt per hyperedge, with round 1 of the repair's
// search: one thread per (copy c, hyperedge i) writes the copy's members of
// i (the stubs at the sorted positions, as k_null_gather) and, when they
// repeat a node, lists i among copy c's kBadLists lists at
// bad + c * bad_stride, in no particular order (a repair round depends only
// on which hyperedges are bad: the partners are drawn by position in the
// list and the union is sorted).  Copy c < R has its own repair workgroup.
__global__ void k_null_deal(uint32_t R, uint32_t E, uint64_t T, const unsigned long long* __restrict__ off,
                            const uint32_t* __restrict__ vals, const uint32_t* __restrict__ stubs,
                            uint32_t* __restrict__ members, RepairScratch sc) {
  const uint64_t n = uint64_t(R) * E;
  for (uint64_t it = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; it < n; it += uint64_t(gridDim.x) * blockDim.x) {
    const uint32_t c = uint32_t(it / E), i = uint32_t(it - uint64_t(c) * E);
    const unsigned long long b = off[i];
    const uint32_t s = uint32_t(off[i + 1] - b);
    const uint64_t base = uint64_t(c) * T;
    uint32_t* m = members + base + b;
    for (uint32_t j = 0; j < s; ++j) m[j] = stubs[vals[base + b + j] - base];
    if (repeats_node(m, s)) {
      const uint64_t list = uint64_t(c) * kBadLists + i % kBadLists;
      sc.bad[uint64_t(c) * sc.bad_stride + (i % kBadLists) * sc.bad_cap + atomicAdd(&sc.counts[list * kBadStride], 1u)] = i;
    }
  }
}

// One workgroup per copy: repair rounds until no hyperedge repeats a node.
// pre: k_null_deal has listed round 1's hyperedges (R <= gridDim.x, so the
// workgroup's copy is its own index).  A round whose chosen list fits the LDS
// sort (2 n_bad <= kLdsBitonic) keeps the list, the pool offsets and, when
// the pool fits too, the pool and its keys in LDS; larger rounds use the
// scratch arrays in device memory (the sort works on either).
__global__ void __launch_bounds__(kThreads) k_null_repair(uint32_t c0, uint32_t R, uint32_t E, uint64_t T,
                                                          const unsigned long long* __restrict__ off,
                                                          uint32_t* __restrict__ members,
                                                          const unsigned long long* __restrict__ seed_p,
                                                          RepairScratch sc, bool pre, uint32_t* __restrict__ failed) {
  __shared__ uint32_t wsum[kWavesPerBlock];
  __shared__ uint32_t lstart[kBadLists + 1];
  __shared__ unsigned long long lk[kLdsBitonic];
  __shared__ uint32_t la[kLdsBitonic], lv[kLdsBitonic];
  __shared__ uint32_t lchosen[kLdsBitonic], lpoff[kLdsBitonic];
  const unsigned long long seed = *seed_p;
  for (uint32_t c = blockIdx.x; c < R; c += gridDim.x) {
    uint32_t* m = members + uint64_t(c) * T;
    uint32_t* bad = sc.bad + uint64_t(blockIdx.x) * sc.bad_stride;
    uint32_t* g_chosen = sc.chosen + uint64_t(blockIdx.x) * sc.chosen_pad;
    unsigned long long* g_key = sc.key + uint64_t(blockIdx.x) * sc.pool_pad;
    uint32_t* g_aux = sc.aux + uint64_t(blockIdx.x) * sc.pool_pad;
    uint32_t* g_val = sc.val + uint64_t(blockIdx.x) * sc.pool_pad;
    uint32_t* g_poff = sc.off + uint64_t(blockIdx.x) * sc.chosen_pad;
    const unsigned long long k1 = (kDomainNull << 32) | (c0 + c);
    // round 1 looks at every hyperedge (pre: k_null_deal did, into lists
    // that are joined here through the chosen scratch); later rounds only at
    // the last pool
    uint32_t n_bad = 0;
    if (pre) {
      if (threadIdx.x == 0) {
        uint32_t at = 0;
        for (uint32_t k = 0; k < kBadLists; ++k) {
          lstart[k] = at;
          at += sc.counts[(uint64_t(c) * kBadLists + k) * kBadStride];
        }
        lstart[kBadLists] = at;
      }
      __syncthreads();
      n_bad = lstart[kBadLists];
      for (uint32_t k = threadIdx.x / kWave; k < kBadLists; k += kWavesPerBlock)
        for (uint32_t j = lstart[k] + (threadIdx.x & (kWave - 1)); j < lstart[k + 1]; j += kWave)
          g_chosen[j] = bad[k * sc.bad_cap + (j - lstart[k])];
      __syncthreads();
      for (uint32_t q = threadIdx.x; q < n_bad; q += kThreads) bad[q] = g_chosen[q];
      __syncthreads();
    } else {
      n_bad = block_compact(E, [&](uint32_t i) {
        return repeats_node(m + off[i], uint32_t(off[i + 1] - off[i]));
      }, bad, wsum);
    }
    int r = 1;
    for (; n_bad > 0 && r <= kMaxRepairRounds; ++r) {
      uint32_t pad = 1;
      while (pad < 2 * n_bad) pad <<= 1;
      const bool small = pad <= kLdsBitonic;   // uniform over the workgroup
      uint32_t* chosen = small ? lchosen : g_chosen;
      uint32_t* poff = small ? lpoff : g_poff;
      unsigned long long* key = small ? lk : g_key;
      uint32_t* aux = small ? la : g_aux;
      uint32_t* tmp = small ? lv : bad;   // (bad is not read again in the round once copied)
      // partners, then the ascending union of bad and partners
      for (uint32_t q = threadIdx.x; q < 2 * n_bad; q += kThreads)
        chosen[q] = q < n_bad ? bad[q]
                              : uint32_t(bounded64(philox4x64_10(q - n_bad, uint64_t(r), 1, 0, seed, k1).v[0], E));
      for (uint32_t q = 2 * n_bad + threadIdx.x; q < pad; q += kThreads) chosen[q] = 0xFFFFFFFFu;
      __syncthreads();
      // sort the 32-bit list with the key and aux arrays (key = value)
      for (uint32_t q = threadIdx.x; q < pad; q += kThreads) {
        key[q] = chosen[q];
        aux[q] = 0;
      }
      __syncthreads();
      block_bitonic(key, aux, nullptr, pad, lk, la, lv);
      for (uint32_t q = threadIdx.x; q < pad; q += kThreads) chosen[q] = uint32_t(key[q]);
      __syncthreads();
      const uint32_t n_ch = block_compact(2 * n_bad, [&](uint32_t q) {
        return q == 0 || chosen[q] != chosen[q - 1];
      }, aux, wsum);
      // aux[0..n_ch) = positions of first copies; gather them (ascending, unique)
      for (uint32_t q = threadIdx.x; q < n_ch; q += kThreads) tmp[q] = chosen[aux[q]];
      __syncthreads();
      for (uint32_t q = threadIdx.x; q < n_ch; q += kThreads) chosen[q] = tmp[q];
      __syncthreads();
      // pool offsets and gather
      uint32_t pool = 0;
      for (uint32_t base = 0; base < n_ch; base += kThreads) {
        const uint32_t q = base + threadIdx.x;
        const uint32_t s = q < n_ch ? uint32_t(off[chosen[q] + 1] - off[chosen[q]]) : 0u;
        uint32_t tot;
        const uint32_t pos = block_exclusive_scan(s, wsum, &tot);
        if (q < n_ch) poff[q] = pool + pos;
        pool += tot;
      }
      __syncthreads();
      if (pool > sc.pool_pad) {
        if (threadIdx.x == 0) atomicOr(failed, 2u);
        break;
      }
      uint32_t ppad = 1;
      while (ppad < pool) ppad <<= 1;
      const bool pool_small = small && ppad <= kLdsBitonic;
      unsigned long long* pkey = pool_small ? lk : g_key;
      uint32_t* paux = pool_small ? la : g_aux;
      uint32_t* pval = pool_small ? lv : g_val;
      for (uint32_t q = threadIdx.x; q < n_ch; q += kThreads) {
        const unsigned long long b = off[chosen[q]];
        const uint32_t s = uint32_t(off[chosen[q] + 1] - b);
        for (uint32_t t = 0; t < s; ++t) pval[poff[q] + t] = m[b + t];
      }
      __syncthreads();
      for (uint32_t t = threadIdx.x; t < ppad; t += kThreads) {
        if (t < pool) {
          pkey[t] = philox4x64_10(t, uint64_t(r), 0, 0, seed, k1).v[0];
          paux[t] = t;
        } else {
          pkey[t] = ~0ull;
          paux[t] = 0xFFFFFFFFu;
          pval[t] = 0;
        }
      }
      __syncthreads();
      block_bitonic(pkey, paux, pval, ppad, lk, la, lv);
      // deal back and find the hyperedges that still repeat a node
      for (uint32_t q = threadIdx.x; q < n_ch; q += kThreads) {
        const unsigned long long b = off[chosen[q]];
        const uint32_t s = uint32_t(off[chosen[q] + 1] - b);
        for (uint32_t t = 0; t < s; ++t) m[b + t] = pval[poff[q] + t];
      }
      __syncthreads();
      n_bad = block_compact(n_ch, [&](uint32_t q) {
        const unsigned long long b = off[chosen[q]];
        return repeats_node(m + b, uint32_t(off[chosen[q] + 1] - b));
      }, paux, wsum);
      for (uint32_t q = threadIdx.x; q < n_bad; q += kThreads) bad[q] = chosen[paux[q]];
      __syncthreads();
    }
    if (n_bad > 0 && threadIdx.x == 0) atomicOr(failed, 1u);
    __syncthreads();
  }
}

__device__ inline double wave_sum_f64(double x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

// z_m over the R copies, fp64, rounded to fp32: one wavefront per class m
// (blockIdx.x), its lanes taking the copies in turn
__global__ void __launch_bounds__(kWave) k_zscore(const int64_t* __restrict__ real, const int64_t* __restrict__ nulls,
                                                  uint32_t R, int n_classes, float* __restrict__ z) {
  const int c = blockIdx.x;
  const uint32_t lane = threadIdx.x;
  double s = 0.0;
  for (uint32_t i = lane; i < R; i += kWave) s += double(nulls[uint64_t(i) * n_classes + c]);
  const double mean = wave_sum_f64(s) / double(R);
  double ss = 0.0;
  for (uint32_t i = lane; i < R; i += kWave) {
    const double d = double(nulls[uint64_t(i) * n_classes + c]) - mean;
    ss += d * d;
  }
  ss = wave_sum_f64(ss);
  if (lane != 0) return;
  const double sd = sqrt(ss / double(R - 1));
  const double x = double(real[c]);
  double out;
  if (sd > 0.0) out = (x - mean) / sd;
  else out = x > mean ? __builtin_huge_val() : (x < mean ? -__builtin_huge_val() : 0.0);
  z[c] = float(out);
}

unsigned grid_for(uint64_t n, unsigned cap = 4096) {
  uint64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return unsigned(g);
}

uint64_t pow2_at_least(uint64_t n) {
  uint64_t p = 1;
  while (p < n) p <<= 1;
  return p;
}

int bits_for(uint64_t n) {
  int b = 1;
  while (b < 64 && (1ull << b) < n) ++b;
  return b;
}

// ---------------------------------------------------------------- batched ingest of the copies
// Every copy has the size sequence of the unique hyperedges of H (offsets
// `off`, E hyperedges, T members).  Index spaces run over (copy, hyperedge);
// per-size outputs of all copies are concatenated copy by copy, and
// incidence indices are positions in those concatenations.  Capacities come
// from H (a copy cannot hold more hyperedges of a size than H), so nothing
// depends on host-side counts.

__global__ void k_b_prepare(uint32_t R, uint32_t E, uint64_t T, const unsigned long long* __restrict__ off,
                            uint32_t* __restrict__ members, unsigned long long* __restrict__ hash) {
  const uint64_t n = uint64_t(R) * E;
  for (uint64_t idx = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < n; idx += uint64_t(gridDim.x) * blockDim.x) {
    const uint64_t c = idx / E, i = idx % E;
    const uint32_t s = uint32_t(off[i + 1] - off[i]);
    if (s < 2 || s > 4) {
      hash[idx] = 0;
      continue;
    }
    uint32_t* m = members + c * T + off[i];
    // the members loaded at once and sorted by a network (padding, above any
    // node id, sorts last)
    uint32_t r[4];
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) r[j] = j < s ? m[j] : 0xFFFFFFFFu;
    constexpr int kNet[5][2] = {{0, 1}, {2, 3}, {0, 2}, {1, 3}, {1, 2}};
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const uint32_t x = r[kNet[q][0]], y = r[kNet[q][1]];
      r[kNet[q][0]] = min(x, y);
      r[kNet[q][1]] = max(x, y);
    }
    unsigned long long h = mix64(0x51ed270b27a3ffb1ull ^ s);
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j)
      if (j < s) {
        m[j] = r[j];
        h = mix64(h ^ (r[j] + 0x9e3779b97f4a7c15ull * (j + 1)));
      }
    hash[idx] = h;
  }
}

__device__ inline bool same_copy_tuple(const uint32_t* mc, const unsigned long long* off, uint32_t a, uint32_t b) {
  const uint32_t sa = uint32_t(off[a + 1] - off[a]);
  if (sa != uint32_t(off[b + 1] - off[b])) return false;
  const uint32_t* x = mc + off[a];
  const uint32_t* y = mc + off[b];
  for (uint32_t j = 0; j < sa; ++j)
    if (x[j] != y[j]) return false;
  return true;
}

__global__ void k_b_dedup(uint32_t R, uint32_t E, uint64_t T, const unsigned long long* __restrict__ off,
                          const uint32_t* __restrict__ members, const unsigned long long* __restrict__ hash,
                          uint32_t* __restrict__ tab, unsigned long long capD) {
  const uint64_t n = uint64_t(R) * E;
  for (uint64_t idx = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < n; idx += uint64_t(gridDim.x) * blockDim.x) {
    const uint64_t c = idx / E;
    const uint32_t i = uint32_t(idx % E);
    const uint32_t s = uint32_t(off[i + 1] - off[i]);
    const unsigned long long hi = hash[idx];   // (loaded with the size)
    if (s < 2 || s > 4) continue;
    uint32_t* t = tab + c * capD;
    const uint32_t* mc = members + c * T;
    unsigned long long pos = hi & (capD - 1);
    while (true) {
      // claim the slot if empty (most are: the table is at most half full)
      const uint32_t cur = atomicCAS(&t[pos], kEmpty32, i);
      if (cur == kEmpty32) break;
      if (hash[c * E + cur] == hi && same_copy_tuple(mc, off, cur, i)) {
        atomicMin(&t[pos], i);
        break;
      }
      pos = (pos + 1) & (capD - 1);
    }
  }
}

__global__ void k_b_first(uint32_t R, uint32_t E, uint64_t T, const unsigned long long* __restrict__ off,
                          const uint32_t* __restrict__ members, const unsigned long long* __restrict__ hash,
                          const uint32_t* __restrict__ tab, unsigned long long capD, uint32_t* f2, uint32_t* f3,
                          uint32_t* f4) {
  const uint64_t n = uint64_t(R) * E;
  for (uint64_t idx = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < n; idx += uint64_t(gridDim.x) * blockDim.x) {
    const uint64_t c = idx / E;
    const uint32_t i = uint32_t(idx % E);
    const uint32_t s = uint32_t(off[i + 1] - off[i]);
    const unsigned long long hi = hash[idx];   // (loaded with the size)
    bool first = false;
    if (s >= 2 && s <= 4) {
      const uint32_t* t = tab + c * capD;
      const uint32_t* mc = members + c * T;
      unsigned long long pos = hi & (capD - 1);
      while (true) {
        const uint32_t cur = t[pos];
        if (cur == kEmpty32) break;
        if (cur == i) {   // the slot of i's tuple, holding i itself
          first = true;
          break;
        }
        if (hash[c * E + cur] == hi && same_copy_tuple(mc, off, cur, i)) {
          first = cur == i;
          break;
        }
        pos = (pos + 1) & (capD - 1);
      }
    }
    f2[idx] = first && s == 2;
    f3[idx] = first && s == 3;
    f4[idx] = first && s == 4;
  }
}

__global__ void k_b_bases(uint32_t R, uint32_t E, const uint32_t* __restrict__ p2, const uint32_t* __restrict__ p3,
                          const uint32_t* __restrict__ p4, const uint32_t* __restrict__ tot, uint32_t* base2,
                          uint32_t* base3, uint32_t* base4) {
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c <= R; c += gridDim.x * blockDim.x) {
    base2[c] = c < R ? p2[uint64_t(c) * E] : tot[0];
    base3[c] = c < R ? p3[uint64_t(c) * E] : tot[1];
    base4[c] = c < R ? p4[uint64_t(c) * E] : tot[2];
  }
}

__global__ void k_b_gather(uint32_t R, uint32_t E, uint64_t T, const unsigned long long* __restrict__ off,
                           const uint32_t* __restrict__ members, const uint32_t* __restrict__ f2,
                           const uint32_t* __restrict__ f3, const uint32_t* __restrict__ f4,
                           const uint32_t* __restrict__ p2, const uint32_t* __restrict__ p3,
                           const uint32_t* __restrict__ p4, uint32_t* e2, uint32_t* e3, uint32_t* e4, uint32_t* copy2,
                           uint32_t* copy3, uint32_t* copy4) {
  const uint64_t n = uint64_t(R) * E;
  for (uint64_t idx = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < n; idx += uint64_t(gridDim.x) * blockDim.x) {
    const uint64_t c = idx / E, i = idx % E;
    const uint32_t* m = members + c * T + off[i];
    if (f2[idx]) {
      const uint64_t q = p2[idx];
      e2[2 * q] = m[0];
      e2[2 * q + 1] = m[1];
      copy2[q] = uint32_t(c);
    } else if (f3[idx]) {
      const uint64_t q = p3[idx];
      for (int j = 0; j < 3; ++j) e3[3 * q + j] = m[j];
      copy3[q] = uint32_t(c);
    } else if (f4[idx]) {
      const uint64_t q = p4[idx];
      for (int j = 0; j < 4; ++j) e4[4 * q + j] = m[j];
      copy4[q] = uint32_t(c);
    }
  }
}

__global__ void k_b_set64(uint64_t cap_items, const uint32_t* __restrict__ total, const uint32_t* __restrict__ e2,
                          const uint32_t* __restrict__ copy2, unsigned long long* slots, unsigned long long cap) {
  const uint64_t n = *total;
  for (uint64_t q = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < n && q < cap_items;
       q += uint64_t(gridDim.x) * blockDim.x) {
    unsigned long long* s = slots + uint64_t(copy2[q]) * cap;
    const unsigned long long key = key2(e2[2 * q], e2[2 * q + 1]);
    unsigned long long pos = mix64(key) & (cap - 1);
    while (atomicCAS(s + pos, kEmpty64, key) != kEmpty64) pos = (pos + 1) & (cap - 1);
  }
}

template <int J>
__global__ void k_b_set128(uint64_t cap_items, const uint32_t* __restrict__ total, const uint32_t* __restrict__ e,
                           const uint32_t* __restrict__ copyj, unsigned long long* slots, unsigned long long cap) {
  const uint64_t n = *total;
  for (uint64_t q = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < n && q < cap_items;
       q += uint64_t(gridDim.x) * blockDim.x) {
    unsigned long long* s = slots + uint64_t(copyj[q]) * 2 * cap;
    const uint32_t* t = e + J * q;
    const Key128 key = (J == 3) ? key3(t[0], t[1], t[2]) : key4(t[0], t[1], t[2], t[3]);
    unsigned long long pos = hash128(key) & (cap - 1);
    while (atomicCAS(s + 2 * pos, kEmpty64, key.hi) != kEmpty64) pos = (pos + 1) & (cap - 1);
    s[2 * pos + 1] = key.lo;
  }
}

__global__ void k_b_pair_keys(uint64_t cap_items, const uint32_t* __restrict__ total, const uint32_t* __restrict__ e2,
                              const uint32_t* __restrict__ copy2, uint32_t N, int B, unsigned long long* keys,
                              uint32_t* vals, uint32_t* deg) {
  const uint64_t n = *total;
  for (uint64_t q = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < cap_items;
       q += uint64_t(gridDim.x) * blockDim.x) {
    vals[2 * q] = 0;
    vals[2 * q + 1] = 0;
    if (q >= n) {
      keys[2 * q] = ~0ull;
      keys[2 * q + 1] = ~0ull;
      continue;
    }
    const unsigned long long c = copy2[q];
    const uint32_t a = e2[2 * q], b = e2[2 * q + 1];
    keys[2 * q] = (c << (2 * B)) | ((unsigned long long)a << B) | b;
    keys[2 * q + 1] = (c << (2 * B)) | ((unsigned long long)b << B) | a;
    atomicAdd(&deg[c * N + a], 1u);
    atomicAdd(&deg[c * N + b], 1u);
  }
}

__global__ void k_b_pair_adj(const unsigned long long* __restrict__ keys, uint64_t n, unsigned long long mask,
                             uint32_t* adj) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
    adj[i] = uint32_t(keys[i] & mask);
}

template <int J>
__global__ void k_b_inc_count(uint64_t cap_items, const uint32_t* __restrict__ total, const uint32_t* __restrict__ e,
                              const uint32_t* __restrict__ copyj, uint32_t N, uint32_t* deg) {
  const uint64_t n = *total;
  for (uint64_t q = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < n && q < cap_items;
       q += uint64_t(gridDim.x) * blockDim.x)
    for (int j = 0; j < J; ++j) atomicAdd(&deg[uint64_t(copyj[q]) * N + e[J * q + j]], 1u);
}

// (with bit rows, oth not null: each entry also gets the hyperedge's other
// members, others3 or others4)
template <int J, typename O>
__global__ void k_b_inc_fill(uint64_t cap_items, const uint32_t* __restrict__ total, const uint32_t* __restrict__ e,
                             const uint32_t* __restrict__ copyj, uint32_t N, uint32_t* cursor, uint32_t* idx,
                             O* __restrict__ oth) {
  const uint64_t n = *total;
  for (uint64_t q = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < n && q < cap_items;
       q += uint64_t(gridDim.x) * blockDim.x) {
    uint32_t m[J], at[J];
    const uint64_t row = uint64_t(copyj[q]) * N;
#pragma unroll
    for (int j = 0; j < J; ++j) m[j] = e[J * q + j];
    // every member's cursor taken before any entry is written, so that the
    // atomics go out together
#pragma unroll
    for (int j = 0; j < J; ++j) at[j] = atomicAdd(&cursor[row + m[j]], 1u);
#pragma unroll
    for (int j = 0; j < J; ++j) {
      idx[at[j]] = uint32_t(q);
      if (oth) {
        if constexpr (J == 3) oth[at[j]] = others3(m, j);
        else oth[at[j]] = others4(m, j);
      }
    }
  }
}

__global__ void k_b_bits(uint64_t cap_items, const uint32_t* __restrict__ total, const uint32_t* __restrict__ e2,
                         const uint32_t* __restrict__ copy2, uint32_t N, uint32_t W, uint32_t* bits) {
  const uint64_t n = *total;
  for (uint64_t q = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < n && q < cap_items;
       q += uint64_t(gridDim.x) * blockDim.x) {
    uint32_t* b = bits + uint64_t(copy2[q]) * N * W;
    const uint32_t u = e2[2 * q], v = e2[2 * q + 1];
    atomicOr(&b[uint64_t(u) * W + (v >> 5)], 1u << (v & 31));
    atomicOr(&b[uint64_t(v) * W + (u >> 5)], 1u << (u & 31));
  }
}

// ---------------------------------------------------------------- persistent counting
// Work is cut into tiles of one phase of one copy: phase 0 = (b) 3-node
// hyperedges (a wavefront per item), phase 1 = (c) pairs (a wavefront per
// item at order 4; a lane per item at order 3), phase 2 = (a) hyperedges of
// size k (a lane per item).  Tiles are ordered phase-major, heaviest phase
// first; every wavefront takes the next tile from an atomic counter until
// none is left, so copies of uneven size share the machine.
struct BatchView {
  const uint32_t *e2, *e3, *e4, *g2_off, *g2_adj, *i3_off, *i3_idx, *i4_off, *i4_idx;
  const uint32_t* i3_oth;
  const unsigned long long* i4_oth;
  unsigned long long *hs2, *hs3, *hs4;
  unsigned long long cap2, cap3, cap4;
  const uint32_t* bits;
  uint32_t W, N;
  const uint32_t *base2, *base3, *base4;
};

__device__ inline View copy_view(const BatchView& b, uint32_t c) {
  View v;
  v.e2 = b.e2;
  v.e3 = b.e3;
  v.e4 = b.e4;
  v.g2_off = b.g2_off + uint64_t(c) * b.N;
  v.g2_adj = b.g2_adj;
  v.i3_off = b.i3_off + uint64_t(c) * b.N;
  v.i3_idx = b.i3_idx;
  v.i4_off = b.i4_off + uint64_t(c) * b.N;
  v.i4_idx = b.i4_idx;
  v.i3_oth = b.i3_oth;
  v.i4_oth = b.i4_oth;
  v.hs2 = Set64{b.hs2 + uint64_t(c) * b.cap2, b.cap2 - 1};
  v.hs3 = Set128{b.hs3 + uint64_t(c) * 2 * b.cap3, b.cap3 - 1};
  v.hs4 = Set128{b.hs4 + uint64_t(c) * 2 * b.cap4, b.cap4 - 1};
  v.bits = b.bits ? b.bits + uint64_t(c) * b.N * b.W : nullptr;
  v.W = b.W;
  v.N = b.N;
  return v;
}

struct Chunks {
  uint32_t per_tile[3];   // items per tile of each phase
};

// Per copy: kMain, kSub and kG2 regions, then the seven identity sums.
constexpr uint32_t kNullHistStride = kIdAcc + 16;

// With the identity route (order 4 with bit rows), phase 1 of a copy takes
// its pairs, then one item per node.
__device__ inline bool batch_ident(const BatchView& b, int k) { return k == 4 && b.bits && use_identities(b.N, b.W); }

__global__ void k_tile_counts(uint32_t R, int k, BatchView b, Chunks ch, uint32_t* counts) {
  for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < 3 * R; s += gridDim.x * blockDim.x) {
    const uint32_t ph = s / R, c = s % R;
    uint32_t items = 0;
    if (ph == 0) items = k == 4 ? b.base3[c + 1] - b.base3[c] : 0;
    if (ph == 1) items = b.base2[c + 1] - b.base2[c] + (batch_ident(b, k) ? b.N : 0u);
    if (ph == 2) items = k == 4 ? b.base4[c + 1] - b.base4[c] : b.base3[c + 1] - b.base3[c];
    counts[s] = (items + ch.per_tile[ph] - 1) / ch.per_tile[ph];
  }
}

__global__ void __launch_bounds__(kThreads) k_null_count(BatchView b, uint32_t R, int k,
                                                         const uint32_t* __restrict__ tile_prefix,
                                                         uint32_t* __restrict__ counter, Chunks ch,
                                                         const uint8_t* __restrict__ lut_g,
                                                         unsigned long long* __restrict__ hist_all) {
  __shared__ uint8_t lut[2048];
  __shared__ unsigned long long wh[kWavesPerBlock][512];
  extern __shared__ uint32_t b4_sets[];   // b4_set_words(W) words per wavefront
  __shared__ uint32_t ylist[kWavesPerBlock][kWave];
  load_lut(lut, lut_g, k == 4 ? 2048 : 16);
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  unsigned long long* h_main = wh[wv];
  unsigned long long* h_sub = wh[wv] + 256;
  const uint32_t total = tile_prefix[3 * R];
  const C4Lanes L = c4_lanes(b.W);
  while (true) {
    uint32_t t = 0;
    if (lane == 0) t = atomicAdd(counter, 1u);
    t = __shfl(t, 0, kWave);
    if (t >= total) break;
    // the slot (phase, copy) whose tile range holds t
    uint32_t lo = 0, hi = 3 * R;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (tile_prefix[mid] <= t) lo = mid; else hi = mid;
    }
    const uint32_t ph = lo / R, c = lo % R;
    const uint32_t first = (t - tile_prefix[lo]) * ch.per_tile[ph];
    const View v = copy_view(b, c);
    unsigned long long* hc = hist_all + uint64_t(c) * kNullHistStride;
    for (uint32_t i = lane; i < 512; i += kWave) wh[wv][i] = 0;
    wave_sync();
    if (ph == 0) {
      const uint32_t n = b.base3[c + 1] - b.base3[c];
      const uint32_t last = min(n, first + ch.per_tile[0]);
      for (uint32_t j = first; j < last; ++j) b4_item(v, b.base3[c] + j, b4_sets + wv * b4_set_words(b.W), lut, h_main, h_sub);
    } else if (ph == 1) {
      const uint32_t n2c = b.base2[c + 1] - b.base2[c];
      const bool id = batch_ident(b, k);
      const uint32_t n = n2c + (id ? b.N : 0u);
      const uint32_t last = min(n, first + ch.per_tile[1]);
      if (id) {
        IdAcc acc;
        id_zero(acc);
        for (uint32_t j = first; j < last; ++j) {
          if (j < n2c) {
            const uint64_t q = b.base2[c] + j;
            id_edge_item(v, b.e2[2 * q], b.e2[2 * q + 1], L, ylist[wv], acc);
          } else {
            id_node_item(v, j - n2c, acc);
          }
        }
        id_flush(acc, hc + kIdAcc);
      } else if (k == 4) {
        if (v.bits) {
          C4Acc acc;
          c4_zero(acc);
          for (uint32_t j = first; j < last; ++j) {
            const uint64_t q = b.base2[c] + j;
            c4_bits_item(v, b.e2[2 * q], b.e2[2 * q + 1], L, ylist[wv], acc, lut, hc + kG2);
          }
          c4_flush(acc, lut, hc + kG2);
        } else {
          for (uint32_t j = first; j < last; ++j) {
            const uint64_t q = b.base2[c] + j;
            c4_hash_item(v, b.e2[2 * q], b.e2[2 * q + 1], lut, h_main);
          }
        }
      } else {
        C3Acc acc{0, 0, 0};
        for (uint32_t j = first + lane; j < last; j += kWave) {
          const uint64_t q = b.base2[c] + j;
          const uint32_t r = b.e2[2 * q], y = b.e2[2 * q + 1];
          if (v.bits) {
            for (uint32_t w = 0; w < v.W; ++w) c3_bits_word(v, r, y, w, acc);
          } else {
            c3_hash_item(v, r, y, acc);
          }
        }
        c3_flush(acc, lut, hc + kG2);
      }
    } else {
      if (k == 4) {
        const uint32_t n = b.base4[c + 1] - b.base4[c];
        const uint32_t last = min(n, first + ch.per_tile[2]);
        for (uint32_t j = first + lane; j < last; j += kWave) {
          const uint64_t q = b.base4[c] + j;
          count_class(lut, h_main, h_sub, a4_pattern(v, b.e4[4 * q], b.e4[4 * q + 1], b.e4[4 * q + 2], b.e4[4 * q + 3]),
                      kPairBits4);
        }
      } else {
        const uint32_t n = b.base3[c + 1] - b.base3[c];
        const uint32_t last = min(n, first + ch.per_tile[2]);
        for (uint32_t j = first + lane; j < last; j += kWave) {
          const uint64_t q = b.base3[c] + j;
          count_class(lut, h_main, h_sub, a3_pattern(v, b.e3[3 * q], b.e3[3 * q + 1], b.e3[3 * q + 2]), kPairBits3);
        }
      }
    }
    wave_sync();
    // wavefront counters -> the copy's counters; the hash-set variant of (c)
    // at order 4 counts G2 shapes in the first half
    const bool g2_in_main = (ph == 1 && k == 4 && !v.bits);
    for (uint32_t i = lane; i < 512; i += kWave) {
      const unsigned long long x = wh[wv][i];
      if (!x) continue;
      if (g2_in_main) {
        if (i < 256) atomicAdd(hc + kG2 + i, x);
      } else {
        atomicAdd(hc + i, x);   // kMain = 0, kSub = 256
      }
    }
    wave_sync();
  }
}

// Order 4 with bit rows, a copy's bit matrix and row starts small enough for
// LDS (null_lds_bytes): a workgroup takes a tile at a time, copies the bit
// matrix and the row starts of the tile's copy into LDS when the copy
// changes, and its wavefronts share the tile's items (every wavefront the
// next of every kWavesPerBlock items; phase 2 one item per thread).  The
// items then read adjacency words and row bounds from LDS rather than L2,
// as the single-graph count does.  Dynamic LDS: the wavefronts' b4 sets,
// then the rows (16-byte aligned) and the three row-start arrays.
__host__ __device__ inline size_t null_lds_table_words(uint32_t N, uint32_t W) {
  return size_t(N) * W + 3 * (size_t(N) + 1);
}
__global__ void __launch_bounds__(kThreads) k_null_count_lds(BatchView b, uint32_t R,
                                                             const uint32_t* __restrict__ tile_prefix,
                                                             uint32_t* __restrict__ counter, Chunks ch,
                                                             const uint8_t* __restrict__ lut_g,
                                                             unsigned long long* __restrict__ hist_all) {
  __shared__ uint8_t lut[2048];
  __shared__ unsigned long long wh[kWavesPerBlock][512];
  extern __shared__ uint32_t dyn_lds[];
  __shared__ uint32_t ylist[kWavesPerBlock][kWave];
  __shared__ uint32_t s_tile;
  load_lut(lut, lut_g, 2048);
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  unsigned long long* h_main = wh[wv];
  unsigned long long* h_sub = wh[wv] + 256;
  uint32_t* sets = dyn_lds + wv * b4_set_words(b.W);
  uint32_t* rows = dyn_lds + kWavesPerBlock * b4_set_words(b.W);
  const uint32_t nw = b.N * b.W;
  uint32_t* offs = rows + nw;
  const uint32_t total = tile_prefix[3 * R];
  const C4Lanes L = c4_lanes(b.W);
  const bool id = batch_ident(b, 4);
  uint32_t loaded = 0xFFFFFFFFu;
  while (true) {
    __syncthreads();   // the previous tile is done with s_tile and the LDS tables
    if (threadIdx.x == 0) s_tile = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t t = s_tile;
    if (t >= total) break;
    // the slot (phase, copy) whose tile range holds t
    uint32_t lo = 0, hi = 3 * R;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (tile_prefix[mid] <= t) lo = mid; else hi = mid;
    }
    const uint32_t ph = lo / R, c = lo % R;
    const uint32_t first = (t - tile_prefix[lo]) * ch.per_tile[ph];
    View v = copy_view(b, c);
    if (c != loaded) {
      const uint4* src = reinterpret_cast<const uint4*>(v.bits);
      uint4* dst = reinterpret_cast<uint4*>(rows);
      for (uint32_t i = threadIdx.x; i < nw / 4; i += kThreads) dst[i] = src[i];
      for (uint32_t i = 4 * (nw / 4) + threadIdx.x; i < nw; i += kThreads) rows[i] = v.bits[i];
      for (uint32_t i = threadIdx.x; i <= b.N; i += kThreads) {
        offs[i] = v.g2_off[i];
        offs[b.N + 1 + i] = v.i3_off[i];
        offs[2 * (b.N + 1) + i] = v.i4_off[i];
      }
      loaded = c;
      __syncthreads();
    }
    v.bits = rows;
    v.g2_off = offs;
    v.i3_off = offs + b.N + 1;
    v.i4_off = offs + 2 * (b.N + 1);
    unsigned long long* hc = hist_all + uint64_t(c) * kNullHistStride;
    for (uint32_t i = lane; i < 512; i += kWave) wh[wv][i] = 0;
    wave_sync();
    if (ph == 0) {
      const uint32_t n = b.base3[c + 1] - b.base3[c];
      const uint32_t last = min(n, first + ch.per_tile[0]);
      for (uint32_t j = first + wv; j < last; j += kWavesPerBlock) b4_item(v, b.base3[c] + j, sets, lut, h_main, h_sub);
    } else if (ph == 1) {
      const uint32_t n2c = b.base2[c + 1] - b.base2[c];
      const uint32_t n = n2c + (id ? b.N : 0u);
      const uint32_t last = min(n, first + ch.per_tile[1]);
      if (id) {
        IdAcc acc;
        id_zero(acc);
        for (uint32_t j = first + wv; j < last; j += kWavesPerBlock) {
          if (j < n2c) {
            const uint64_t q = b.base2[c] + j;
            id_edge_item(v, b.e2[2 * q], b.e2[2 * q + 1], L, ylist[wv], acc);
          } else {
            id_node_item(v, j - n2c, acc);
          }
        }
        id_flush(acc, hc + kIdAcc);
      } else {
        C4Acc acc;
        c4_zero(acc);
        for (uint32_t j = first + wv; j < last; j += kWavesPerBlock) {
          const uint64_t q = b.base2[c] + j;
          c4_bits_item(v, b.e2[2 * q], b.e2[2 * q + 1], L, ylist[wv], acc, lut, hc + kG2);
        }
        c4_flush(acc, lut, hc + kG2);
      }
    } else {
      const uint32_t n = b.base4[c + 1] - b.base4[c];
      const uint32_t last = min(n, first + ch.per_tile[2]);
      for (uint32_t j = first + threadIdx.x; j < last; j += kThreads) {
        const uint64_t q = b.base4[c] + j;
        count_class(lut, h_main, h_sub, a4_pattern(v, b.e4[4 * q], b.e4[4 * q + 1], b.e4[4 * q + 2], b.e4[4 * q + 3]),
                    kPairBits4);
      }
    }
    wave_sync();
    for (uint32_t i = lane; i < 512; i += kWave) {
      const unsigned long long x = wh[wv][i];
      if (x) atomicAdd(hc + i, x);   // kMain = 0, kSub = 256
    }
  }
}

struct ClassMaskB {
  unsigned long long w[4];
};

__global__ void k_b_combine(const unsigned long long* __restrict__ hist_all, int n_classes, ClassMaskB pairs_only,
                            IdShapes sh, int64_t* __restrict__ counts) {
  const uint32_t c = blockIdx.x;
  const int m = threadIdx.x;
  if (m >= n_classes) return;
  const unsigned long long* h = hist_all + uint64_t(c) * kNullHistStride;
  unsigned long long v = h[kMain + m];
  if ((pairs_only.w[m >> 6] >> (m & 63)) & 1ull)
    v += (sh.on ? id_shape_count(h + kIdAcc, sh, m) : h[kG2 + m]) - h[kSub + m];
  counts[uint64_t(c) * n_classes + m] = int64_t(v);
}

}  // namespace

// ---------------------------------------------------------------- plan
struct NullPlan {
  int k = 0;
  int model = HM_NULL_STUBS, sweeps = 0;
  uint32_t* cfg_tmp = nullptr;   // working slots of the configuration model (R x T)
  uint32_t R = 0, E = 0, N = 0;
  uint64_t T = 0, n2H = 0, n3H = 0, n4H = 0;
  int B = 0;
  uint32_t W = 0;
  bool use_bits = false;
  unsigned long long capD = 0, cap2 = 0, cap3 = 0, cap4 = 0;
  Chunks chunks{{4, 4, 256}};
  uint32_t repair_blocks = 0;
  // buffers
  unsigned long long* seed = nullptr;
  uint32_t* members = nullptr;
  unsigned long long *skeys = nullptr, *skeys_tmp = nullptr;
  uint32_t *svals = nullptr, *svals_tmp = nullptr;
  uint32_t* sort_ws = nullptr;
  RepairScratch rs{};
  uint32_t* failed = nullptr;
  unsigned long long* hash = nullptr;
  uint32_t* dtab = nullptr;
  uint32_t *f2 = nullptr, *f3 = nullptr, *f4 = nullptr, *p2 = nullptr, *p3 = nullptr, *p4 = nullptr;
  uint32_t* tot = nullptr;
  uint32_t* scan_ws = nullptr;
  uint32_t *base2 = nullptr, *base3 = nullptr, *base4 = nullptr;
  uint32_t *e2 = nullptr, *e3 = nullptr, *e4 = nullptr, *copy2 = nullptr, *copy3 = nullptr, *copy4 = nullptr;
  unsigned long long *hs2 = nullptr, *hs3 = nullptr, *hs4 = nullptr;
  unsigned long long *pkeys = nullptr, *pkeys_tmp = nullptr;
  uint32_t *pvals = nullptr, *pvals_tmp = nullptr;
  uint32_t *deg = nullptr, *cursor = nullptr;
  uint32_t *g2_off = nullptr, *g2_adj = nullptr, *i3_off = nullptr, *i3_idx = nullptr, *i4_off = nullptr,
           *i4_idx = nullptr;
  uint32_t* i3_oth = nullptr;          // with bit rows
  unsigned long long* i4_oth = nullptr;
  uint32_t* bits = nullptr;
  unsigned long long* hist_all = nullptr;
  uint32_t *tile_counts = nullptr, *tile_prefix = nullptr, *tile_counter = nullptr;
  int64_t *real = nullptr, *nulls = nullptr;
  float* z = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<void*> allocs;

  template <typename T>
  int get(T** p, uint64_t n) {
    void* q = nullptr;
    HM_TRY(dalloc(&q, size_t(n ? n : 1) * sizeof(T)));
    allocs.push_back(q);
    *p = static_cast<T*>(q);
    return HM_OK;
  }
  ~NullPlan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipDeviceSynchronize();
    for (void* p : allocs) dfree(p);
  }
};

void destroy_null_plan(NullPlan* p) { delete p; }

namespace {

BatchView batch_view(const NullPlan& P) {
  BatchView b;
  b.e2 = P.e2;
  b.e3 = P.e3;
  b.e4 = P.e4;
  b.g2_off = P.g2_off;
  b.g2_adj = P.g2_adj;
  b.i3_off = P.i3_off;
  b.i3_idx = P.i3_idx;
  b.i4_off = P.i4_off;
  b.i4_idx = P.i4_idx;
  b.i3_oth = P.i3_oth;
  b.i4_oth = P.i4_oth;
  b.hs2 = P.hs2;
  b.hs3 = P.hs3;
  b.hs4 = P.hs4;
  b.cap2 = P.cap2;
  b.cap3 = P.cap3;
  b.cap4 = P.cap4;
  b.bits = P.use_bits ? P.bits : nullptr;
  b.W = P.W;
  b.N = P.N;
  b.base2 = P.base2;
  b.base3 = P.base3;
  b.base4 = P.base4;
  return b;
}

int make_plan(const hm_graph* H, int k, uint32_t R, int model, int sweeps, NullPlan** out) {
  NullPlan* P = new (std::nothrow) NullPlan();
  if (!P) {
    set_error("host allocation failed");
    return HM_ENOMEM;
  }
  P->k = k;
  P->R = R;
  P->model = model;
  P->sweeps = sweeps;
  P->E = uint32_t(H->n_unique);
  P->T = H->n_unique_members;
  P->N = H->n_nodes;
  P->n2H = H->n_by_size[2];
  P->n3H = H->n_by_size[3];
  P->n4H = H->n_by_size[4];
  P->B = bits_for(P->N);
  P->use_bits = H->bits != nullptr;
  P->W = P->use_bits ? H->words : 0;
  P->capD = pow2_capacity(P->E);
  P->cap2 = pow2_capacity(P->n2H);
  P->cap3 = pow2_capacity(P->n3H);
  P->cap4 = pow2_capacity(P->n4H);
  const uint64_t RT = uint64_t(R) * P->T, RE = uint64_t(R) * P->E, RN = uint64_t(R) * P->N;
  const uint64_t m2 = uint64_t(R) * P->n2H, m3 = uint64_t(R) * P->n3H, m4 = uint64_t(R) * P->n4H;
  auto fail = [&](int rc) {
    delete P;
    return rc;
  };
  if (RT >= 0xFFFFFFFFull || RE >= 0xFFFFFFFFull || 2 * m2 >= 0xFFFFFFFFull || RN >= 0xFFFFFFFFull ||
      2 * P->B + bits_for(R) > 64) {
    set_error("null batch too large (%u copies)", R);
    return fail(HM_EUNSUPPORTED);
  }
  int rc = HM_OK;
#define GET(ptr, n) \
  if (rc == HM_OK) rc = P->get(&(ptr), (n))
  GET(P->seed, 1);
  GET(P->members, RT);
  if (model == HM_NULL_CONFIG) GET(P->cfg_tmp, RT);
  GET(P->skeys, RT);
  GET(P->skeys_tmp, RT);
  GET(P->svals, RT);
  GET(P->svals_tmp, RT);
  const uint64_t sort_words = std::max(radix_ws_words(RT), radix_ws_words(2 * m2 + 2));
  GET(P->sort_ws, sort_words);
  P->repair_blocks = R < 256 ? R : 256;
  P->rs.chosen_pad = pow2_at_least(2ull * P->E + 2);
  P->rs.pool_pad = pow2_at_least(P->T + 1);
  P->rs.bad_cap = (P->E + kBadLists - 1) / kBadLists;
  P->rs.bad_stride = uint64_t(kBadLists) * P->rs.bad_cap;
  GET(P->rs.bad, uint64_t(P->repair_blocks) * P->rs.bad_stride + 1);
  GET(P->rs.counts, uint64_t(P->repair_blocks) * kBadLists * kBadStride);
  GET(P->rs.chosen, uint64_t(P->repair_blocks) * P->rs.chosen_pad);
  GET(P->rs.off, uint64_t(P->repair_blocks) * P->rs.chosen_pad);
  GET(P->rs.key, uint64_t(P->repair_blocks) * P->rs.pool_pad);
  GET(P->rs.aux, uint64_t(P->repair_blocks) * P->rs.pool_pad);
  GET(P->rs.val, uint64_t(P->repair_blocks) * P->rs.pool_pad);
  GET(P->failed, 1);
  GET(P->hash, RE);
  GET(P->dtab, uint64_t(R) * P->capD);
  GET(P->f2, RE);
  GET(P->f3, RE);
  GET(P->f4, RE);
  GET(P->p2, RE);
  GET(P->p3, RE);
  GET(P->p4, RE);
  GET(P->tot, 4);
  GET(P->scan_ws, std::max(scan_ws_words(RE), scan_ws_words(RN + 1)) + scan_ws_words(3ull * R + 1));
  GET(P->base2, uint64_t(R) + 1);
  GET(P->base3, uint64_t(R) + 1);
  GET(P->base4, uint64_t(R) + 1);
  GET(P->e2, 2 * m2);
  GET(P->e3, 3 * m3);
  GET(P->e4, 4 * m4);
  GET(P->copy2, m2);
  GET(P->copy3, m3);
  GET(P->copy4, m4);
  GET(P->hs2, uint64_t(R) * P->cap2);
  GET(P->hs3, uint64_t(R) * 2 * P->cap3);
  GET(P->hs4, uint64_t(R) * 2 * P->cap4);
  GET(P->pkeys, 2 * m2 + 2);
  GET(P->pkeys_tmp, 2 * m2 + 2);
  GET(P->pvals, 2 * m2 + 2);
  GET(P->pvals_tmp, 2 * m2 + 2);
  GET(P->deg, RN);
  GET(P->cursor, RN);
  GET(P->g2_off, RN + 1);
  GET(P->g2_adj, 2 * m2 + 2);
  GET(P->i3_off, RN + 1);
  GET(P->i3_idx, 3 * m3);
  GET(P->i4_off, RN + 1);
  GET(P->i4_idx, 4 * m4);
  if (P->use_bits) {
    GET(P->bits, RN * P->W);
    GET(P->i3_oth, 3 * m3);
    GET(P->i4_oth, 4 * m4);
  }
  GET(P->hist_all, uint64_t(R) * kNullHistStride);
  GET(P->tile_counts, 3ull * R + 1);
  GET(P->tile_prefix, 3ull * R + 1);
  GET(P->tile_counter, 1);
  const int C = class_tables().n_classes[k];
  GET(P->real, uint64_t(C));
  GET(P->nulls, uint64_t(R) * C);
  GET(P->z, uint64_t(C));
#undef GET
  if (rc != HM_OK) return fail(rc);
  *out = P;
  return HM_OK;
}

// P.svals := for each copy in turn, its `per` items in the order of their
// words (see k_order_keys); no allocation, no sync.
int enqueue_order(NullPlan& P, uint64_t n, uint64_t per, uint64_t round, unsigned long long domain, uint32_t c0,
                  hipStream_t st) {
  k_order_keys<<<grid_for(n), 256, 0, st>>>(c0, P.R, per, round, domain, P.seed, P.skeys, P.svals);
  HM_HIP(hipGetLastError());
  HM_TRY(radix_sort_ws(P.skeys, P.svals, P.skeys_tmp, P.svals_tmp, n, 32 + bits_for(P.R), P.sort_ws, st));
  k_fix_ties<<<grid_for(n), 256, 0, st>>>(P.skeys, P.svals, n, per, round, c0, domain, P.seed);
  HM_HIP(hipGetLastError());
  return HM_OK;
}

// Stub matching of copies c0 .. c0+R-1 into P.members (no allocation, no sync).
int enqueue_stubs(const hm_graph* H, NullPlan& P, uint32_t c0, hipStream_t st) {
  const uint64_t n = uint64_t(P.R) * P.T;
  if (n == 0) return HM_OK;
  HM_TRY(enqueue_order(P, n, P.T, 0, kDomainNull, c0, st));
  HM_TRY(fill_u32(P.failed, 0, 1, st));
  const bool pre = P.R <= P.repair_blocks;
  if (pre) {
    HM_TRY(fill_u32(P.rs.counts, 0, uint64_t(P.R) * kBadLists * kBadStride, st));
    k_null_deal<<<grid_for(uint64_t(P.R) * P.E), 256, 0, st>>>(P.R, P.E, P.T, H->all_off, P.svals, H->all_members,
                                                                P.members, P.rs);
  } else {
    k_null_gather<<<grid_for(n), 256, 0, st>>>(P.svals, n, P.T, H->all_members, P.members);
  }
  HM_HIP(hipGetLastError());
  k_null_repair<<<P.repair_blocks, kThreads, 0, st>>>(c0, P.R, P.E, P.T, H->all_off, P.members, P.seed, P.rs, pre,
                                                      P.failed);
  HM_HIP(hipGetLastError());
  return HM_OK;
}

// Configuration-model copies c0 .. c0+R-1 into P.members (no allocation, no
// sync): every copy starts from the input and runs P.sweeps rounds of
// pairwise reshuffles.
int enqueue_config(const hm_graph* H, NullPlan& P, uint32_t c0, hipStream_t st) {
  const uint64_t n = uint64_t(P.R) * P.T, ne = uint64_t(P.R) * P.E;
  HM_TRY(fill_u32(P.failed, 0, 1, st));
  if (n == 0) return HM_OK;
  k_cfg_init<<<grid_for(n), 256, 0, st>>>(P.R, P.T, H->all_members, P.members);
  HM_HIP(hipGetLastError());
  if (P.E < 2) return HM_OK;
  for (int r = 0; r < P.sweeps; ++r) {
    HM_TRY(enqueue_order(P, ne, P.E, uint64_t(r), kDomainConfig, c0, st));
    k_cfg_pairs<<<grid_for(uint64_t(P.R) * (P.E / 2)), 256, 0, st>>>(c0, P.R, P.E, P.T, uint32_t(r), P.seed, P.svals,
                                                                    H->all_off, P.members, P.cfg_tmp);
    HM_HIP(hipGetLastError());
  }
  return HM_OK;
}

// Batched ingest of the copies in P.members.
int enqueue_ingest(const hm_graph* H, NullPlan& P, hipStream_t st) {
  const uint32_t R = P.R, E = P.E, N = P.N;
  const uint64_t RE = uint64_t(R) * E, RN = uint64_t(R) * N;
  const uint64_t m2 = uint64_t(R) * P.n2H, m3 = uint64_t(R) * P.n3H, m4 = uint64_t(R) * P.n4H;
  k_b_prepare<<<grid_for(RE), 256, 0, st>>>(R, E, P.T, H->all_off, P.members, P.hash);
  HM_TRY(fill_u32(P.dtab, kEmpty32, uint64_t(R) * P.capD, st));
  k_b_dedup<<<grid_for(RE), 256, 0, st>>>(R, E, P.T, H->all_off, P.members, P.hash, P.dtab, P.capD);
  k_b_first<<<grid_for(RE), 256, 0, st>>>(R, E, P.T, H->all_off, P.members, P.hash, P.dtab, P.capD, P.f2, P.f3,
                                          P.f4);
  HM_HIP(hipGetLastError());
  HM_TRY(scan_u32_ws(P.f2, P.p2, RE, P.tot + 0, P.scan_ws, st));
  HM_TRY(scan_u32_ws(P.f3, P.p3, RE, P.tot + 1, P.scan_ws, st));
  HM_TRY(scan_u32_ws(P.f4, P.p4, RE, P.tot + 2, P.scan_ws, st));
  k_b_bases<<<grid_for(R + 1), 256, 0, st>>>(R, E, P.p2, P.p3, P.p4, P.tot, P.base2, P.base3, P.base4);
  k_b_gather<<<grid_for(RE), 256, 0, st>>>(R, E, P.T, H->all_off, P.members, P.f2, P.f3, P.f4, P.p2, P.p3, P.p4, P.e2,
                                           P.e3, P.e4, P.copy2, P.copy3, P.copy4);
  HM_HIP(hipGetLastError());
  HM_TRY(fill_u64(P.hs2, kEmpty64, uint64_t(R) * P.cap2, st));
  HM_TRY(fill_u64(P.hs3, kEmpty64, uint64_t(R) * 2 * P.cap3, st));
  HM_TRY(fill_u64(P.hs4, kEmpty64, uint64_t(R) * 2 * P.cap4, st));
  if (m2) k_b_set64<<<grid_for(m2), 256, 0, st>>>(m2, P.tot + 0, P.e2, P.copy2, P.hs2, P.cap2);
  if (m3) k_b_set128<3><<<grid_for(m3), 256, 0, st>>>(m3, P.tot + 1, P.e3, P.copy3, P.hs3, P.cap3);
  if (m4) k_b_set128<4><<<grid_for(m4), 256, 0, st>>>(m4, P.tot + 2, P.e4, P.copy4, P.hs4, P.cap4);
  HM_HIP(hipGetLastError());
  // pairwise graph rows (ascending) of every copy
  HM_TRY(fill_u32(P.deg, 0, RN, st));
  if (m2) {
    k_b_pair_keys<<<grid_for(m2), 256, 0, st>>>(m2, P.tot + 0, P.e2, P.copy2, N, P.B, P.pkeys, P.pvals, P.deg);
    HM_HIP(hipGetLastError());
    HM_TRY(radix_sort_ws(P.pkeys, P.pvals, P.pkeys_tmp, P.pvals_tmp, 2 * m2, 2 * P.B + bits_for(R), P.sort_ws, st));
    k_b_pair_adj<<<grid_for(2 * m2), 256, 0, st>>>(P.pkeys, 2 * m2, (1ull << P.B) - 1, P.g2_adj);
    HM_HIP(hipGetLastError());
  }
  HM_TRY(scan_u32_ws(P.deg, P.g2_off, RN, P.g2_off + RN, P.scan_ws, st));
  // incident 3- and 4-node hyperedges
  HM_TRY(fill_u32(P.deg, 0, RN, st));
  if (m3) k_b_inc_count<3><<<grid_for(m3), 256, 0, st>>>(m3, P.tot + 1, P.e3, P.copy3, N, P.deg);
  HM_HIP(hipGetLastError());
  HM_TRY(scan_u32_ws(P.deg, P.i3_off, RN, P.i3_off + RN, P.scan_ws, st));
  HM_TRY(copy_u32(P.i3_off, P.cursor, RN, st));
  if (m3) k_b_inc_fill<3><<<grid_for(m3), 256, 0, st>>>(m3, P.tot + 1, P.e3, P.copy3, N, P.cursor, P.i3_idx, P.i3_oth);
  HM_TRY(fill_u32(P.deg, 0, RN, st));
  if (m4) k_b_inc_count<4><<<grid_for(m4), 256, 0, st>>>(m4, P.tot + 2, P.e4, P.copy4, N, P.deg);
  HM_HIP(hipGetLastError());
  HM_TRY(scan_u32_ws(P.deg, P.i4_off, RN, P.i4_off + RN, P.scan_ws, st));
  HM_TRY(copy_u32(P.i4_off, P.cursor, RN, st));
  if (m4) k_b_inc_fill<4><<<grid_for(m4), 256, 0, st>>>(m4, P.tot + 2, P.e4, P.copy4, N, P.cursor, P.i4_idx, P.i4_oth);
  HM_HIP(hipGetLastError());
  if (P.use_bits) {
    HM_TRY(fill_u32(P.bits, 0, RN * P.W, st));
    if (m2) k_b_bits<<<grid_for(m2), 256, 0, st>>>(m2, P.tot + 0, P.e2, P.copy2, N, P.W, P.bits);
    HM_HIP(hipGetLastError());
  }
  return HM_OK;
}

// Workgroups of the persistent counting kernel: as many as are resident at
// once with `lds` bytes of dynamic LDS each, at most four per CU.
unsigned persistent_grid(size_t lds) {
  int dev = 0, cus = 256, per_cu = 2;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_null_count, kThreads, lds) != hipSuccess) per_cu = 2;
  per_cu = per_cu < 1 ? 1 : (per_cu > 4 ? 4 : per_cu);
  return unsigned(cus > 0 ? cus : 256) * unsigned(per_cu);
}

// Workgroups of k_null_count_lds resident at once, at most four per CU: the
// register and wave limits from the occupancy query without LDS, the LDS
// limit from the CU's LDS size (static plus `lds` dynamic bytes per
// workgroup).  More workgroups than fit only wait for the first to finish:
// the count claims its tiles until none is left.
unsigned persistent_grid_lds(size_t lds) {
  int dev = 0, cus = 256, per_cu = 1, lds_cu = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
  }
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_null_count_lds, kThreads, 0) != hipSuccess) per_cu = 1;
  hipFuncAttributes attr{};
  size_t per_wg = lds;
  if (hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(k_null_count_lds)) == hipSuccess)
    per_wg += attr.sharedSizeBytes;
  (void)hipGetLastError();
  if (lds_cu > 0 && per_wg > 0) per_cu = std::min<int>(per_cu, int(size_t(lds_cu) / per_wg));
  per_cu = per_cu < 1 ? 1 : (per_cu > 4 ? 4 : per_cu);
  return unsigned(cus > 0 ? cus : 256) * unsigned(per_cu);
}

// Whether the batch counts with k_null_count_lds (order 4, bit rows, a copy's
// tables in at most kNullLdsMaxBytes), and its dynamic LDS.
constexpr size_t kNullLdsMaxBytes = 48 * 1024;
bool null_lds(const NullPlan& P) {
  return P.k == 4 && P.use_bits && null_lds_table_words(P.N, P.W) * 4 <= kNullLdsMaxBytes;
}
size_t null_lds_bytes(const NullPlan& P) {
  return (size_t(kWavesPerBlock) * b4_set_words(P.W) + null_lds_table_words(P.N, P.W)) * 4;
}

int enqueue_count(const hm_graph* H, NullPlan& P, const Chunks& ch, hipStream_t st) {
  const uint8_t *lut4 = nullptr, *lut3 = nullptr;
  HM_TRY(device_luts(H->device, &lut4, &lut3));
  const BatchView bv = batch_view(P);
  const uint32_t R = P.R;
  k_tile_counts<<<grid_for(3ull * R), 256, 0, st>>>(R, P.k, bv, ch, P.tile_counts);
  HM_HIP(hipGetLastError());
  HM_TRY(scan_u32_ws(P.tile_counts, P.tile_prefix, 3ull * R, P.tile_prefix + 3ull * R, P.scan_ws, st));
  HM_TRY(fill_u64(P.hist_all, 0, uint64_t(R) * kNullHistStride, st));
  HM_TRY(fill_u32(P.tile_counter, 0, 1, st));
  if (null_lds(P)) {
    const size_t lds = null_lds_bytes(P);
    k_null_count_lds<<<persistent_grid_lds(lds), kThreads, lds, st>>>(bv, R, P.tile_prefix, P.tile_counter, ch, lut4,
                                                                      P.hist_all);
  } else {
    const size_t lds = (P.k == 4 && bv.bits) ? size_t(kWavesPerBlock) * b4_set_words(bv.W) * 4 : 0;
    k_null_count<<<persistent_grid(lds), kThreads, lds, st>>>(bv, R, P.k, P.tile_prefix, P.tile_counter, ch,
                                                         P.k == 4 ? lut4 : lut3, P.hist_all);
  }
  HM_HIP(hipGetLastError());
  const ClassTables& t = class_tables();
  ClassMaskB pairs_only{{0, 0, 0, 0}};
  for (int c = 0; c < t.n_classes[P.k]; ++c)
    if (t.maxcard[P.k][c] == 2) pairs_only.w[c >> 6] |= 1ull << (c & 63);
  k_b_combine<<<R, 256, 0, st>>>(P.hist_all, t.n_classes[P.k], pairs_only,
                                 id_shapes(P.k == 4 && P.use_bits && use_identities(P.N, P.W)), P.nulls);
  HM_HIP(hipGetLastError());
  return HM_OK;
}

// The seed-dependent part of a call (the real counts in P.real do not depend
// on it and are counted once, before capture).
int enqueue_copies(const hm_graph* H, NullPlan& P, uint32_t c0, hipStream_t st) {
  return P.model == HM_NULL_CONFIG ? enqueue_config(H, P, c0, st) : enqueue_stubs(H, P, c0, st);
}

int enqueue_all(const hm_graph* H, NullPlan& P, hipStream_t st) {
  HM_TRY(enqueue_copies(H, P, 0, st));
  HM_TRY(enqueue_ingest(H, P, st));
  HM_TRY(enqueue_count(H, P, P.chunks, st));
  const int C = class_tables().n_classes[P.k];
  k_zscore<<<C, kWave, 0, st>>>(P.real, P.nulls, P.R, C, P.z);
  HM_HIP(hipGetLastError());
  return HM_OK;
}

// ---------------------------------------------------------------- autotuner
// Items per tile of phases (b) and (c) are picked by timing the persistent
// counting kernel on the ingested copies; choices are cached per device and
// shape signature for the life of the process.
using TuneKey = std::tuple<int, int, uint32_t, uint32_t, uint64_t, uint64_t, uint64_t, uint32_t, bool>;
std::mutex g_tune_mu;
std::map<TuneKey, Chunks> g_tuned;

int autotune(const hm_graph* H, NullPlan& P, hipStream_t st) {
  const TuneKey key{H->device, P.k, P.R, P.N, P.n2H, P.n3H, P.n4H, P.E, P.use_bits};
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      P.chunks = it->second;
      return HM_OK;
    }
  }
  // items per tile: per wavefront, or with k_null_count_lds per workgroup
  // (its kWavesPerBlock wavefronts share a tile)
  static const uint32_t cand_wave[] = {1, 2, 4, 8, 16};
  static const uint32_t cand_block[] = {64, 128, 256, 512, 1024};
  const uint32_t* cand_b = null_lds(P) ? cand_block : cand_wave;
  const uint32_t* cand_c = cand_b;
  hipEvent_t e0, e1;
  HM_HIP(hipEventCreate(&e0));
  HM_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  Chunks best_ch = P.chunks;
  for (int ib = 0; ib < 5; ++ib)
    for (int ic = 0; ic < 5; ++ic) {
      const uint32_t cb = cand_b[ib], cc = cand_c[ic];
      Chunks ch{{cb, cc, P.k == 4 ? 256u : 1024u}};
      if (P.k == 3) ch.per_tile[1] = 64 * cc;
      float total = 0.f;
      for (int rep = 0; rep < 2; ++rep) {
        HM_HIP(hipEventRecord(e0, st));
        HM_TRY(enqueue_count(H, P, ch, st));
        HM_HIP(hipEventRecord(e1, st));
        HM_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        HM_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (rep) total += ms;
      }
      if (total < best) {
        best = total;
        best_ch = ch;
      }
      if (P.k == 3) break;   // order 3: one lane per pair; only (c) chunking matters
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  P.chunks = best_ch;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tuned[key] = best_ch;
  return HM_OK;
}

}  // namespace

// Generate copies [c0, c0 + R) into members (R x T, device), synchronously.
int null_copies(const hm_graph* H, uint32_t c0, uint32_t R, uint64_t seed, uint32_t* members, hipStream_t st,
                int model, int sweeps) {
  note_use(H, st);
  if (H->n_unique_members == 0 || R == 0) return HM_OK;
  NullPlan P;
  P.model = model;
  P.sweeps = sweeps;
  P.R = R;
  P.E = uint32_t(H->n_unique);
  P.T = H->n_unique_members;
  const uint64_t RT = uint64_t(R) * P.T;
  if (RT >= 0xFFFFFFFFull) {
    set_error("null batch too large");
    return HM_EUNSUPPORTED;
  }
  HM_TRY(P.get(&P.seed, 1));
  HM_TRY(P.get(&P.skeys, RT));
  HM_TRY(P.get(&P.skeys_tmp, RT));
  HM_TRY(P.get(&P.svals, RT));
  HM_TRY(P.get(&P.svals_tmp, RT));
  HM_TRY(P.get(&P.sort_ws, radix_ws_words(RT)));
  P.repair_blocks = R < 256 ? R : 256;
  P.rs.chosen_pad = pow2_at_least(2ull * P.E + 2);
  P.rs.pool_pad = pow2_at_least(P.T + 1);
  P.rs.bad_cap = (P.E + kBadLists - 1) / kBadLists;
  P.rs.bad_stride = uint64_t(kBadLists) * P.rs.bad_cap;
  HM_TRY(P.get(&P.rs.bad, uint64_t(P.repair_blocks) * P.rs.bad_stride + 1));
  HM_TRY(P.get(&P.rs.counts, uint64_t(P.repair_blocks) * kBadLists * kBadStride));
  HM_TRY(P.get(&P.rs.chosen, uint64_t(P.repair_blocks) * P.rs.chosen_pad));
  HM_TRY(P.get(&P.rs.off, uint64_t(P.repair_blocks) * P.rs.chosen_pad));
  HM_TRY(P.get(&P.rs.key, uint64_t(P.repair_blocks) * P.rs.pool_pad));
  HM_TRY(P.get(&P.rs.aux, uint64_t(P.repair_blocks) * P.rs.pool_pad));
  HM_TRY(P.get(&P.rs.val, uint64_t(P.repair_blocks) * P.rs.pool_pad));
  HM_TRY(P.get(&P.failed, 1));
  if (model == HM_NULL_CONFIG) HM_TRY(P.get(&P.cfg_tmp, RT));
  P.members = members;
  unsigned long long s = seed;
  HM_HIP(hipMemcpyAsync(P.seed, &s, sizeof(s), hipMemcpyHostToDevice, st));
  HM_TRY(enqueue_copies(H, P, c0, st));
  uint32_t host_failed = 0;
  HM_HIP(hipMemcpyAsync(&host_failed, P.failed, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HM_HIP(hipStreamSynchronize(st));
  if (host_failed) {
    set_error("stub matching: a hyperedge still repeats a node after %d repair rounds", kMaxRepairRounds);
    return HM_EINVAL;
  }
  return HM_OK;
}

int count_nulls_impl(hm_graph* H, int k, uint32_t R, int model, int sweeps, uint64_t seed, int64_t* real,
                     int64_t* nulls, float* z, hipStream_t st) {
  note_use(H, st);
  const int C = class_tables().n_classes[k];
  const uint8_t *lut4 = nullptr, *lut3 = nullptr;
  HM_TRY(device_luts(H->device, &lut4, &lut3));
  if (H->n_unique == 0) {   // nothing to randomise: every count is zero
    if (real) HM_TRY(count_exact_impl(H, k, real, st));
    HM_TRY(fill_u64(reinterpret_cast<unsigned long long*>(nulls), 0, uint64_t(R) * C, st));
    if (z) HM_TRY(fill_u32(reinterpret_cast<uint32_t*>(z), 0, uint64_t(C), st));
    HM_HIP(hipStreamSynchronize(st));
    return HM_OK;
  }
  NullPlan* P = H->null_plan;
  if (P && (P->k != k || P->R != R || P->model != model || P->sweeps != sweeps)) {
    destroy_null_plan(P);
    H->null_plan = P = nullptr;
  }
  if (!P) {
    HM_TRY(make_plan(H, k, R, model, sweeps, &P));
    H->null_plan = P;
    // first run outside a graph: the real counts, then ingest the copies once
    // and tune the tile sizes
    HM_TRY(count_exact_impl(H, k, P->real, st));
    unsigned long long s0 = seed;
    HM_HIP(hipMemcpyAsync(P->seed, &s0, sizeof(s0), hipMemcpyHostToDevice, st));
    HM_TRY(enqueue_copies(H, *P, 0, st));
    HM_TRY(enqueue_ingest(H, *P, st));
    HM_TRY(autotune(H, *P, st));
    // capture the whole pipeline once; later calls replay it
    hipStream_t cs = nullptr;
    HM_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    capture_begin();
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    int rc = e == hipSuccess ? enqueue_all(H, *P, cs) : HM_EDEVICE;
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &g);
    capture_end();
    if (rc == HM_OK && e2 != hipSuccess) rc = HM_EDEVICE;
    if (rc == HM_OK && hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0) != hipSuccess) rc = HM_EDEVICE;
    P->graph = g;
    (void)hipStreamDestroy(cs);
    if (rc != HM_OK) {
      if (rc == HM_EDEVICE) set_error("capturing the null-model pipeline failed");
      destroy_null_plan(P);
      H->null_plan = nullptr;
      return rc;
    }
  }
  unsigned long long s = seed;
  HM_HIP(hipMemcpyAsync(P->seed, &s, sizeof(s), hipMemcpyHostToDevice, st));
  {
    ProfileScope ps("null_pipeline_graph", st);
    HM_HIP(hipGraphLaunch(P->exec, st));
  }
  if (real) HM_TRY(copy_u64(reinterpret_cast<const unsigned long long*>(P->real), reinterpret_cast<unsigned long long*>(real), uint64_t(C), st));
  HM_TRY(copy_u64(reinterpret_cast<const unsigned long long*>(P->nulls), reinterpret_cast<unsigned long long*>(nulls), uint64_t(R) * C, st));
  if (z) HM_TRY(copy_u32(reinterpret_cast<const uint32_t*>(P->z), reinterpret_cast<uint32_t*>(z), uint64_t(C), st));
  uint32_t host_failed = 0;
  HM_HIP(hipMemcpyAsync(&host_failed, P->failed, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HM_HIP(hipStreamSynchronize(st));
  if (host_failed) {
    set_error("stub matching: a hyperedge still repeats a node after %d repair rounds", kMaxRepairRounds);
    return HM_EINVAL;
  }
  return HM_OK;
}

int null_tuned_chunks(const hm_graph* H, uint32_t* out3) {
  if (!H->null_plan) return HM_EINVAL;
  for (int i = 0; i < 3; ++i) out3[i] = H->null_plan->chunks.per_tile[i];
  return HM_OK;
}

}  // namespace hm

extern "C" {

static int null_model_args(int model, int sweeps) {
  if (model != HM_NULL_STUBS && model != HM_NULL_CONFIG) {
    hm::set_error("unknown null model %d", model);
    return HM_EINVAL;
  }
  if (model == HM_NULL_CONFIG && (sweeps < 1 || sweeps > 4096)) {
    hm::set_error("sweeps must be in [1, 4096] for the configuration model");
    return HM_EINVAL;
  }
  return HM_OK;
}

int hm_null_export_model(const hm_graph* H, int model, int sweeps, uint64_t seed, uint32_t copy, uint32_t* members,
                         uint64_t* offsets) {
  try {
    if (!H || !members || !offsets) {
      hm::set_error("NULL argument to hm_null_export_model");
      return HM_EINVAL;
    }
    HM_TRY(null_model_args(model, sweeps));
    const uint64_t T = H->n_unique_members;
    void* buf = nullptr;
    HM_TRY(hm::dalloc(&buf, T * sizeof(uint32_t) + 4));
    int rc = hm::null_copies(H, copy, 1, seed, static_cast<uint32_t*>(buf), nullptr, model,
                             model == HM_NULL_CONFIG ? sweeps : 0);
    if (rc == HM_OK && T) {
      if (hipMemcpy(members, buf, T * sizeof(uint32_t), hipMemcpyDeviceToHost) != hipSuccess) rc = HM_EDEVICE;
    }
    if (rc == HM_OK &&
        hipMemcpy(offsets, H->all_off, (H->n_unique + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost) != hipSuccess)
      rc = HM_EDEVICE;
    (void)hipDeviceSynchronize();
    hm::dfree(buf);
    return rc;
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_null_export(const hm_graph* H, uint64_t seed, uint32_t copy, uint32_t* members, uint64_t* offsets) {
  try {
    return hm_null_export_model(H, HM_NULL_STUBS, 0, seed, copy, members, offsets);
  } catch (...) {
    return hm::api_failure();
  }
}

int count_nulls_model(const hm_graph* H, int k, int n_rand, int model, int sweeps, uint64_t seed, int64_t* real,
                      int64_t* nulls, float* z, void* stream) {
  try {
    if (!H || !nulls) {
      hm::set_error("NULL argument to count_nulls");
      return HM_EINVAL;
    }
    HM_TRY(null_model_args(model, sweeps));
    if (k != 3 && k != 4) {
      hm::set_error("order %d is not supported (3 or 4)", k);
      return HM_EUNSUPPORTED;
    }
    if (n_rand < 2 || n_rand > 65535) {
      hm::set_error("n_rand must be in [2, 65535]");
      return HM_EINVAL;
    }
    return hm::count_nulls_impl(const_cast<hm_graph*>(H), k, uint32_t(n_rand), model,
                                model == HM_NULL_CONFIG ? sweeps : 0, seed, real, nulls, z,
                                static_cast<hipStream_t>(stream));
  } catch (...) {
    return hm::api_failure();
  }
}

int count_nulls(const hm_graph* H, int k, int n_rand, uint64_t seed, int64_t* real, int64_t* nulls, float* z,
                void* stream) {
  try {
    return count_nulls_model(H, k, n_rand, HM_NULL_STUBS, 0, seed, real, nulls, z, stream);
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_motif_profile(const double* real, const double* nulls, int n_rand, int n_classes, double eps, double* delta,
                     double* sp, void* stream) {
  try {
    if (!real || !nulls || (!delta && !sp)) {
      hm::set_error("NULL argument to hm_motif_profile");
      return HM_EINVAL;
    }
    if (n_rand < 1 || n_classes < 1 || n_classes > 65536 || !(eps >= 0.0)) {
      hm::set_error("hm_motif_profile needs n_rand >= 1, 1 <= n_classes <= 65536 and eps >= 0");
      return HM_EINVAL;
    }
    hm::k_motif_profile<<<1, 256, 0, static_cast<hipStream_t>(stream)>>>(real, nulls, uint32_t(n_rand), n_classes, eps,
                                                                         delta, sp);
    HM_HIP(hipGetLastError());
    return HM_OK;
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_stratum_search(const hm_graph* H, int k, uint64_t S, const double* ratio3, int n3, const double* ratio4, int n4,
                      int reps, uint64_t seed, const double* nulls, int n_rand, const double* exact_profile, double eps,
                      double* rho, void* stream) {
  try {
    if (!H || !ratio3 || !nulls || !exact_profile || !rho || (k == 4 && !ratio4)) {
      hm::set_error("NULL argument to hm_stratum_search");
      return HM_EINVAL;
    }
    if (k != 3 && k != 4) {
      hm::set_error("order %d is not supported (3 or 4)", k);
      return HM_EUNSUPPORTED;
    }
    if (k == 3) n4 = 1;
    if (S == 0 || S >= (1ull << 31) || n3 < 1 || n4 < 1 || uint64_t(n3) * n4 > 4096 || reps < 1 || reps > 1024 ||
        n_rand < 1 || !(eps >= 0.0)) {
      hm::set_error("hm_stratum_search: bad sizes (S, grid, reps or n_rand)");
      return HM_EINVAL;
    }
    for (int i = 0; i < n3; ++i)
      if (!(ratio3[i] >= 0.0)) {
        hm::set_error("stratum ratios must be >= 0");
        return HM_EINVAL;
      }
    for (int i = 0; k == 4 && i < n4; ++i)
      if (!(ratio4[i] >= 0.0)) {
        hm::set_error("stratum ratios must be >= 0");
        return HM_EINVAL;
      }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int C = hm::class_tables().n_classes[k];
    const uint64_t cells = uint64_t(n3) * n4;
    std::vector<void*> bufs;
    struct Free {
      std::vector<void*>& b;
      hipStream_t st;
      ~Free() { hm::dfree_on(b.data(), b.size(), st); }
    } release{bufs, st};
    auto get = [&](void** p, size_t bytes) {
      int rc = hm::dalloc(p, bytes);
      if (rc == HM_OK) bufs.push_back(*p);
      return rc;
    };
    void *est_p = nullptr, *estd_p = nullptr, *delta_p = nullptr, *q_p = nullptr;
    HM_TRY(get(&est_p, sizeof(float) * C));
    HM_TRY(get(&estd_p, sizeof(double) * C));
    HM_TRY(get(&delta_p, sizeof(double) * C));
    HM_TRY(get(&q_p, sizeof(double) * 3 * cells * reps));
    float* est = static_cast<float*>(est_p);
    double* estd = static_cast<double*>(estd_p);
    double* delta = static_cast<double*>(delta_p);
    double* q = static_cast<double*>(q_p);
    for (int i = 0; i < n3; ++i)
      for (int j = 0; j < n4; ++j) {
        // S_2 : S_3 : S_4 = 1 : ratio3 : ratio4 with S_2 + S_3 + S_4 = S
        const double r3 = ratio3[i], r4 = k == 4 ? ratio4[j] : 0.0;
        uint64_t Sj[5] = {0, 0, 0, 0, 0};
        Sj[2] = uint64_t(std::llround(double(S) / (1.0 + r3 + r4)));
        Sj[3] = std::min<uint64_t>(S - Sj[2], uint64_t(std::llround(r3 * double(Sj[2]))));
        Sj[4] = k == 4 ? S - Sj[2] - Sj[3] : 0;
        if (k == 3) Sj[3] = S - Sj[2];
        for (int r = 0; r < reps; ++r) {
          const uint64_t cell = uint64_t(i) * n4 + j;
          HM_TRY(hm::sampled_with_sizes(H, k, Sj, seed + uint64_t(r), est, nullptr, st));
          hm::k_f32_to_f64<<<1, 256, 0, st>>>(est, C, estd);
          hm::k_motif_profile<<<1, 256, 0, st>>>(estd, nulls, uint32_t(n_rand), C, eps, delta, nullptr);
          hm::k_profile_quality<<<1, 256, 0, st>>>(delta, exact_profile, C, q + 3 * (cell * reps + r));
          HM_HIP(hipGetLastError());
        }
      }
    std::vector<double> host(3 * cells * reps);
    HM_HIP(hipMemcpyAsync(host.data(), q, sizeof(double) * host.size(), hipMemcpyDeviceToHost, st));
    HM_HIP(hipStreamSynchronize(st));
    for (uint64_t c = 0; c < cells; ++c) {
      double s = 0.0;
      for (int r = 0; r < reps; ++r) s += host[3 * (c * reps + r)];
      rho[c] = s / double(reps);
    }
    return HM_OK;
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_profile_quality(const double* est, const double* exact, int n_classes, double* out3, void* stream) {
  try {
    if (!est || !exact || !out3) {
      hm::set_error("NULL argument to hm_profile_quality");
      return HM_EINVAL;
    }
    if (n_classes < 1 || n_classes > 65536) {
      hm::set_error("n_classes must be in [1, 65536]");
      return HM_EINVAL;
    }
    hm::k_profile_quality<<<1, 256, 0, static_cast<hipStream_t>(stream)>>>(est, exact, n_classes, out3);
    HM_HIP(hipGetLastError());
    return HM_OK;
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_null_tile_sizes(const hm_graph* H, uint32_t* out3) {
  try {
    if (!H || !out3) {
      hm::set_error("NULL argument");
      return HM_EINVAL;
    }
    if (hm::null_tuned_chunks(H, out3) != HM_OK) {
      hm::set_error("count_nulls has not run on this graph");
      return HM_EINVAL;
    }
    return HM_OK;
  } catch (...) {
    return hm::api_failure();
  }
}

}  // extern "C"
