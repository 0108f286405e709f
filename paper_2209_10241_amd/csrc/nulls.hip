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
#include <vector>

#include "hm_device.h"

namespace hm {

int count_exact_impl(const hm_graph* H, int k, int64_t* counts, hipStream_t st);

namespace {

constexpr int kMaxRepairRounds = 64;

__global__ void k_null_keys(uint32_t c0, uint32_t R, uint64_t T, unsigned long long seed, unsigned long long* keys,
                            uint32_t* vals) {
  const uint64_t n = uint64_t(R) * T;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x) {
    const uint64_t c = i / T, t = i % T;
    keys[i] = philox4x64_10(t, 0, 0, 0, seed, (kDomainNull << 32) | (c0 + c)).v[0];
    vals[i] = uint32_t(i);
  }
}

__global__ void k_copy_of(const uint32_t* __restrict__ vals, uint64_t n, uint64_t T, unsigned long long* keys) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
    keys[i] = vals[i] / T;
}

__global__ void k_null_gather(const uint32_t* __restrict__ vals, uint64_t n, uint64_t T,
                              const uint32_t* __restrict__ stubs, uint32_t* __restrict__ members) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x) {
    const uint64_t c = i / T;
    members[i] = stubs[vals[i] - c * T];
  }
}

// ---------------------------------------------------------------- block helpers
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* wsum, uint32_t* total) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, kWave);
    if (lane >= d) x += y;
  }
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
template <typename F>
__device__ uint32_t block_compact(uint32_t n, F flag, uint32_t* out, uint32_t* wsum) {
  uint32_t count = 0;
  for (uint32_t base = 0; base < n; base += kThreads) {
    const uint32_t i = base + threadIdx.x;
    const bool f = i < n && flag(i);
    uint32_t tot;
    const uint32_t pos = block_exclusive_scan(f ? 1u : 0u, wsum, &tot);
    if (f) out[count + pos] = i;
    count += tot;
  }
  __syncthreads();
  return count;
}

// Ascending bitonic sort of n_pad (a power of two) (key, aux) pairs in
// device memory by one workgroup; ties are broken by aux.
__device__ void block_bitonic(unsigned long long* key, uint32_t* aux, uint32_t* val, uint32_t n_pad) {
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

struct RepairScratch {
  uint32_t* bad;                 // E
  uint32_t* chosen;              // 2E padded to a power of two
  unsigned long long* key;       // pool keys, padded
  uint32_t* aux;                 // pool positions
  uint32_t* val;                 // pool nodes
  uint32_t* off;                 // pool offsets per chosen hyperedge
  uint64_t chosen_pad;           // capacity of chosen (power of two)
  uint64_t pool_pad;             // capacity of the pool arrays (power of two)
};

// One workgroup per copy: repair rounds until no hyperedge repeats a node.
__global__ void __launch_bounds__(kThreads) k_null_repair(uint32_t c0, uint32_t R, uint32_t E, uint64_t T,
                                                          const unsigned long long* __restrict__ off,
                                                          uint32_t* __restrict__ members, unsigned long long seed,
                                                          RepairScratch sc, uint32_t* __restrict__ failed) {
  __shared__ uint32_t wsum[kWavesPerBlock];
  for (uint32_t c = blockIdx.x; c < R; c += gridDim.x) {
    uint32_t* m = members + uint64_t(c) * T;
    uint32_t* bad = sc.bad + uint64_t(blockIdx.x) * E;
    uint32_t* chosen = sc.chosen + uint64_t(blockIdx.x) * sc.chosen_pad;
    unsigned long long* key = sc.key + uint64_t(blockIdx.x) * sc.pool_pad;
    uint32_t* aux = sc.aux + uint64_t(blockIdx.x) * sc.pool_pad;
    uint32_t* val = sc.val + uint64_t(blockIdx.x) * sc.pool_pad;
    uint32_t* poff = sc.off + uint64_t(blockIdx.x) * sc.chosen_pad;
    const unsigned long long k1 = (kDomainNull << 32) | (c0 + c);
    // round 1 looks at every hyperedge; later rounds only at the last pool
    uint32_t n_bad = block_compact(E, [&](uint32_t i) {
      return repeats_node(m + off[i], uint32_t(off[i + 1] - off[i]));
    }, bad, wsum);
    int r = 1;
    for (; n_bad > 0 && r <= kMaxRepairRounds; ++r) {
      // partners, then the ascending union of bad and partners
      for (uint32_t q = threadIdx.x; q < 2 * n_bad; q += kThreads)
        chosen[q] = q < n_bad ? bad[q]
                              : uint32_t(bounded64(philox4x64_10(q - n_bad, uint64_t(r), 1, 0, seed, k1).v[0], E));
      uint32_t pad = 1;
      while (pad < 2 * n_bad) pad <<= 1;
      for (uint32_t q = 2 * n_bad + threadIdx.x; q < pad; q += kThreads) chosen[q] = 0xFFFFFFFFu;
      __syncthreads();
      // sort the 32-bit list with the pool arrays as scratch (key = value)
      for (uint32_t q = threadIdx.x; q < pad; q += kThreads) {
        key[q] = chosen[q];
        aux[q] = 0;
      }
      __syncthreads();
      block_bitonic(key, aux, nullptr, pad);
      for (uint32_t q = threadIdx.x; q < pad; q += kThreads) chosen[q] = uint32_t(key[q]);
      __syncthreads();
      const uint32_t n_ch = block_compact(2 * n_bad, [&](uint32_t q) {
        return q == 0 || chosen[q] != chosen[q - 1];
      }, aux, wsum);
      // aux[0..n_ch) = positions of first copies; gather them (ascending, unique)
      for (uint32_t q = threadIdx.x; q < n_ch; q += kThreads) bad[q] = chosen[aux[q]];
      __syncthreads();
      for (uint32_t q = threadIdx.x; q < n_ch; q += kThreads) chosen[q] = bad[q];
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
      for (uint32_t q = threadIdx.x; q < n_ch; q += kThreads) {
        const unsigned long long b = off[chosen[q]];
        const uint32_t s = uint32_t(off[chosen[q] + 1] - b);
        for (uint32_t t = 0; t < s; ++t) val[poff[q] + t] = m[b + t];
      }
      uint32_t ppad = 1;
      while (ppad < pool) ppad <<= 1;
      __syncthreads();
      for (uint32_t t = threadIdx.x; t < ppad; t += kThreads) {
        if (t < pool) {
          key[t] = philox4x64_10(t, uint64_t(r), 0, 0, seed, k1).v[0];
          aux[t] = t;
        } else {
          key[t] = ~0ull;
          aux[t] = 0xFFFFFFFFu;
          val[t] = 0;
        }
      }
      __syncthreads();
      block_bitonic(key, aux, val, ppad);
      // deal back and find the hyperedges that still repeat a node
      for (uint32_t q = threadIdx.x; q < n_ch; q += kThreads) {
        const unsigned long long b = off[chosen[q]];
        const uint32_t s = uint32_t(off[chosen[q] + 1] - b);
        for (uint32_t t = 0; t < s; ++t) m[b + t] = val[poff[q] + t];
      }
      __syncthreads();
      n_bad = block_compact(n_ch, [&](uint32_t q) {
        const unsigned long long b = off[chosen[q]];
        return repeats_node(m + b, uint32_t(off[chosen[q] + 1] - b));
      }, aux, wsum);
      for (uint32_t q = threadIdx.x; q < n_bad; q += kThreads) bad[q] = chosen[aux[q]];
      __syncthreads();
    }
    if (n_bad > 0 && threadIdx.x == 0) atomicOr(failed, 1u);
    __syncthreads();
  }
}

// z_m over the R copies, fp64, rounded to fp32
__global__ void k_zscore(const int64_t* __restrict__ real, const int64_t* __restrict__ nulls, uint32_t R,
                         int n_classes, float* __restrict__ z) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_classes) return;
  double s = 0.0;
  for (uint32_t i = 0; i < R; ++i) s += double(nulls[uint64_t(i) * n_classes + c]);
  const double mean = s / double(R);
  double ss = 0.0;
  for (uint32_t i = 0; i < R; ++i) {
    const double d = double(nulls[uint64_t(i) * n_classes + c]) - mean;
    ss += d * d;
  }
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

struct NullBuffers {
  std::vector<void*> ptrs;
  ~NullBuffers() {
    for (void* p : ptrs) dfree(p);
  }
  template <typename T>
  int get(T** p, uint64_t n) {
    void* q = nullptr;
    HM_TRY(dalloc(&q, size_t(n ? n : 1) * sizeof(T)));
    ptrs.push_back(q);
    *p = static_cast<T*>(q);
    return HM_OK;
  }
};

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

}  // namespace

// Generate copies [c0, c0 + R) into members (R x T, device).
int null_copies(const hm_graph* H, uint32_t c0, uint32_t R, uint64_t seed, uint32_t* members, hipStream_t st) {
  const uint64_t T = H->n_unique_members;
  const uint32_t E = uint32_t(H->n_unique);
  if (T == 0 || R == 0) return HM_OK;
  const uint64_t n = uint64_t(R) * T;
  if (n >= 0xFFFFFFFFull) {
    set_error("null batch of %llu stubs is too large", (unsigned long long)n);
    return HM_EUNSUPPORTED;
  }
  NullBuffers b;
  unsigned long long *keys, *keys_tmp;
  uint32_t *vals, *vals_tmp, *failed;
  HM_TRY(b.get(&keys, n));
  HM_TRY(b.get(&keys_tmp, n));
  HM_TRY(b.get(&vals, n));
  HM_TRY(b.get(&vals_tmp, n));
  HM_TRY(b.get(&failed, 1));
  // round 0: stable sort by key within each copy (key sort, then a stable sort by copy)
  k_null_keys<<<grid_for(n), 256, 0, st>>>(c0, R, T, seed, keys, vals);
  HM_HIP(hipGetLastError());
  HM_TRY(radix_sort_pairs(keys, vals, keys_tmp, vals_tmp, n, 64, st));
  if (R > 1) {
    k_copy_of<<<grid_for(n), 256, 0, st>>>(vals, n, T, keys);
    HM_HIP(hipGetLastError());
    HM_TRY(radix_sort_pairs(keys, vals, keys_tmp, vals_tmp, n, bits_for(R), st));
  }
  k_null_gather<<<grid_for(n), 256, 0, st>>>(vals, n, T, H->all_members, members);
  HM_HIP(hipGetLastError());
  // repair rounds, one workgroup per copy
  const uint32_t blocks = R < 256 ? R : 256;
  RepairScratch sc;
  sc.chosen_pad = pow2_at_least(2ull * E + 2);
  sc.pool_pad = pow2_at_least(T + 1);
  HM_TRY(b.get(&sc.bad, uint64_t(blocks) * E + 1));
  HM_TRY(b.get(&sc.chosen, uint64_t(blocks) * sc.chosen_pad));
  HM_TRY(b.get(&sc.off, uint64_t(blocks) * sc.chosen_pad));
  HM_TRY(b.get(&sc.key, uint64_t(blocks) * sc.pool_pad));
  HM_TRY(b.get(&sc.aux, uint64_t(blocks) * sc.pool_pad));
  HM_TRY(b.get(&sc.val, uint64_t(blocks) * sc.pool_pad));
  HM_TRY(fill_u32(failed, 0, 1, st));
  k_null_repair<<<blocks, kThreads, 0, st>>>(c0, R, E, T, H->all_off, members, seed, sc, failed);
  HM_HIP(hipGetLastError());
  uint32_t host_failed = 0;
  HM_HIP(hipMemcpyAsync(&host_failed, failed, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HM_HIP(hipStreamSynchronize(st));
  if (host_failed) {
    set_error("stub matching: a hyperedge still repeats a node after %d repair rounds", kMaxRepairRounds);
    return HM_EINVAL;
  }
  return HM_OK;
}

}  // namespace hm

extern "C" {

int hm_null_export(const hm_graph* H, uint64_t seed, uint32_t copy, uint32_t* members, uint64_t* offsets) {
  if (!H || !members || !offsets) {
    hm::set_error("NULL argument to hm_null_export");
    return HM_EINVAL;
  }
  const uint64_t T = H->n_unique_members;
  void* buf = nullptr;
  HM_TRY(hm::dalloc(&buf, T * sizeof(uint32_t) + 4));
  int rc = hm::null_copies(H, copy, 1, seed, static_cast<uint32_t*>(buf), nullptr);
  if (rc == HM_OK && T) {
    if (hipMemcpy(members, buf, T * sizeof(uint32_t), hipMemcpyDeviceToHost) != hipSuccess) rc = HM_EDEVICE;
  }
  if (rc == HM_OK &&
      hipMemcpy(offsets, H->all_off, (H->n_unique + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost) != hipSuccess)
    rc = HM_EDEVICE;
  (void)hipDeviceSynchronize();
  hm::dfree(buf);
  return rc;
}

int count_nulls(const hm_graph* H, int k, int n_rand, uint64_t seed, int64_t* real, int64_t* nulls, float* z,
                void* stream) {
  if (!H || !nulls) {
    hm::set_error("NULL argument to count_nulls");
    return HM_EINVAL;
  }
  if (k != 3 && k != 4) {
    hm::set_error("order %d is not supported (3 or 4)", k);
    return HM_EUNSUPPORTED;
  }
  if (n_rand < 2 || n_rand > 65535) {
    hm::set_error("n_rand must be in [2, 65535]");
    return HM_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int C = hm_num_classes(k);
  const uint64_t T = H->n_unique_members;
  hm::NullBuffers b;
  int64_t* real_buf = real;
  if (!real_buf) HM_TRY(b.get(&real_buf, uint64_t(C)));
  HM_TRY(hm::count_exact_impl(H, k, real_buf, st));
  uint32_t* members = nullptr;
  HM_TRY(b.get(&members, uint64_t(n_rand) * T + 1));
  HM_TRY(hm::null_copies(H, 0, uint32_t(n_rand), seed, members, st));
  for (int c = 0; c < n_rand; ++c) {
    hm_graph* G = nullptr;
    HM_TRY(hm_graph_create(members + uint64_t(c) * T, reinterpret_cast<const uint64_t*>(H->all_off), H->n_unique,
                           H->n_nodes, HM_MEM_DEVICE, stream, &G));
    int rc = hm::count_exact_impl(G, k, nulls + uint64_t(c) * C, st);
    if (rc == HM_OK && hipStreamSynchronize(st) != hipSuccess) rc = HM_EDEVICE;
    hm_graph_destroy(G);
    if (rc != HM_OK) return rc;
  }
  if (z) {
    hm::k_zscore<<<1, 256, 0, st>>>(real_buf, nulls, uint32_t(n_rand), C, z);
    HM_HIP(hipGetLastError());
  }
  HM_HIP(hipStreamSynchronize(st));
  return HM_OK;
}

}  // extern "C"
