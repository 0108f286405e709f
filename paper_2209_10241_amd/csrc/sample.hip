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

#include "hm_b4.h"

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

// j = 4: the sampled 4-node hyperedge is the only candidate set.
__global__ void __launch_bounds__(kThreads) k_sample_j4(const uint32_t* __restrict__ idx, uint64_t S,
                                                        const uint32_t* __restrict__ e4, uint64_t n4, Set64 hs2,
                                                        Set128 hs3, const uint32_t* __restrict__ bits, uint32_t W,
                                                        const uint8_t* __restrict__ lut_g,
                                                        unsigned long long* __restrict__ hist,
                                                        unsigned long long* __restrict__ ps) {
  __shared__ uint8_t lut[2048];
  __shared__ unsigned long long h_lds[256];
  load_lut(lut, lut_g, 2048);
  h_lds[threadIdx.x] = 0;
  __syncthreads();
  for (uint64_t s = uint64_t(blockIdx.x) * kThreads + threadIdx.x; s < S; s += uint64_t(gridDim.x) * kThreads) {
    const uint64_t i = idx[s];
    if (i >= n4) continue;
    unsigned long long* h = ps ? ps + s * 256 : h_lds;
    const uint32_t a = e4[4 * i], b = e4[4 * i + 1], c = e4[4 * i + 2], d = e4[4 * i + 3];
    uint32_t p = 1u << 10;
    p |= pair_bit(hs2, bits, W, a, b) << 0;
    p |= pair_bit(hs2, bits, W, a, c) << 1;
    p |= pair_bit(hs2, bits, W, b, c) << 2;
    p |= uint32_t(set128_has(hs3, key3(a, b, c))) << 3;
    p |= pair_bit(hs2, bits, W, a, d) << 4;
    p |= pair_bit(hs2, bits, W, b, d) << 5;
    p |= uint32_t(set128_has(hs3, key3(a, b, d))) << 6;
    p |= pair_bit(hs2, bits, W, c, d) << 7;
    p |= uint32_t(set128_has(hs3, key3(a, c, d))) << 8;
    p |= uint32_t(set128_has(hs3, key3(b, c, d))) << 9;
    atomicAdd(&h[lut[p]], 1ull);
  }
  __syncthreads();
  flush(h_lds, hist + kRaw, 256);
}

// j = 3 at order 4: the neighbourhood of the sampled 3-node hyperedge.
__global__ void __launch_bounds__(kThreads) k_sample_j3_bits(
    const uint32_t* __restrict__ idx, uint64_t S, const uint32_t* __restrict__ e3, uint64_t n3,
    const uint32_t* __restrict__ e4, const uint32_t* __restrict__ i3_off, const uint32_t* __restrict__ i3_idx,
    const uint32_t* __restrict__ i4_off, const uint32_t* __restrict__ i4_idx, const uint32_t* __restrict__ bits,
    uint32_t W, const uint8_t* __restrict__ lut_g, unsigned long long* __restrict__ hist,
    unsigned long long* __restrict__ ps) {
  __shared__ uint8_t lut[2048];
  __shared__ unsigned long long h[256];
  __shared__ B4Scratch scratch[kWavesPerBlock];
  load_lut(lut, lut_g, 2048);
  h[threadIdx.x] = 0;
  __syncthreads();
  const int wv = threadIdx.x / kWave;
  const uint64_t wave = uint64_t(blockIdx.x) * kWavesPerBlock + wv;
  const uint64_t n_waves = uint64_t(gridDim.x) * kWavesPerBlock;
  for (uint64_t s = wave; s < S; s += n_waves) {
    const uint64_t i = idx[s];
    if (i >= n3) continue;
    b4_edge_bits<false>(e3[3 * i], e3[3 * i + 1], e3[3 * i + 2], e3, e4, i3_off, i3_idx, i4_off, i4_idx, bits, W,
                        scratch[wv], lut, ps ? ps + s * 256 : h, nullptr);
  }
  __syncthreads();
  flush(h, hist + kRaw, 256);
}

__global__ void __launch_bounds__(kThreads) k_sample_j3_hash(
    const uint32_t* __restrict__ idx, uint64_t S, const uint32_t* __restrict__ e3, uint64_t n3,
    const uint32_t* __restrict__ g2_off, const uint32_t* __restrict__ g2_adj, const uint32_t* __restrict__ i3_off,
    const uint32_t* __restrict__ i3_idx, Set64 hs2, Set128 hs3, Set128 hs4, const uint8_t* __restrict__ lut_g,
    unsigned long long* __restrict__ hist, unsigned long long* __restrict__ ps) {
  __shared__ uint8_t lut[2048];
  __shared__ unsigned long long h[256];
  load_lut(lut, lut_g, 2048);
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t wave = uint64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
  const uint64_t n_waves = uint64_t(gridDim.x) * kWavesPerBlock;
  for (uint64_t s = wave; s < S; s += n_waves) {
    const uint64_t i = idx[s];
    if (i >= n3) continue;
    b4_edge_hash<false>(e3[3 * i], e3[3 * i + 1], e3[3 * i + 2], e3, g2_off, g2_adj, i3_off, i3_idx, hs2, hs3, hs4,
                        lut, ps ? ps + s * 256 : h, nullptr);
  }
  __syncthreads();
  flush(h, hist + kRaw, 256);
}

// Row-major index of the pair (p < q) among n items: row p starts at
// p*n - p*(p+1)/2.
__device__ inline void pair_from_index(uint64_t t, uint64_t n, uint32_t& p, uint32_t& q) {
  const double b = double(2 * n - 1);
  double r = (b - sqrt(b * b - 8.0 * double(t))) * 0.5;
  uint64_t pp = r < 0.0 ? 0 : uint64_t(r);
  if (pp > n - 2) pp = n - 2;
  auto start = [n](uint64_t x) { return x * n - x * (x + 1) / 2; };
  while (pp > 0 && start(pp) > t) --pp;
  while (pp + 1 < n - 1 && start(pp + 1) <= t) ++pp;
  p = uint32_t(pp);
  q = uint32_t(t - start(pp) + pp + 1);
}

// j = 2 at order 4: the sampled pair e = {u, w}; the other two nodes x, y make
// e u {x, y} connected through pairs (a larger hyperedge would exceed e).
// L lists the neighbours of u then those of w; a position is valid when its
// node is neither u nor w and, for w's part, not also a neighbour of u, so A
// = the valid nodes, each once.  Either both x and y lie in A (a pair of valid
// positions p < q) or x lies in A and y is a neighbour of x outside A u e.
// One workgroup per sample.
__device__ inline uint32_t nodeL(const uint32_t* g2_adj, uint32_t ub, uint32_t du, uint32_t wb, uint32_t p) {
  return p < du ? g2_adj[ub + p] : g2_adj[wb + (p - du)];
}

__device__ inline void j2_candidate(uint32_t u, uint32_t w, uint32_t x, uint32_t y, const Set64& hs2,
                                    const Set128& hs3, const Set128& hs4, const uint32_t* bits, uint32_t W,
                                    const uint8_t* lut, unsigned long long* h) {
  uint32_t t0 = u, t1 = w, t2 = x;
  sort3(t0, t1, t2);
  if (set128_has(hs3, key3(t0, t1, t2))) return;
  t0 = u; t1 = w; t2 = y;
  sort3(t0, t1, t2);
  if (set128_has(hs3, key3(t0, t1, t2))) return;
  t0 = u; t1 = x; t2 = y;
  sort3(t0, t1, t2);
  if (set128_has(hs3, key3(t0, t1, t2))) return;
  t0 = w; t1 = x; t2 = y;
  sort3(t0, t1, t2);
  if (set128_has(hs3, key3(t0, t1, t2))) return;
  uint32_t q[4] = {u, w, x, y};
  for (int i = 1; i < 4; ++i) {
    const uint32_t k = q[i];
    int j = i - 1;
    while (j >= 0 && q[j] > k) { q[j + 1] = q[j]; --j; }
    q[j + 1] = k;
  }
  if (set128_has(hs4, key4(q[0], q[1], q[2], q[3]))) return;
  // local positions u=0, w=1, x=2, y=3
  const uint32_t p = 1u | (pair_bit(hs2, bits, W, u, x) << 1) | (pair_bit(hs2, bits, W, w, x) << 2) |
                     (pair_bit(hs2, bits, W, u, y) << 4) | (pair_bit(hs2, bits, W, w, y) << 5) |
                     (pair_bit(hs2, bits, W, x, y) << 7);
  const uint8_t cls = lut[p];
  if (cls != 0xFF) atomicAdd(&h[cls], 1ull);
}

__global__ void __launch_bounds__(kThreads) k_sample_j2_k4(
    const uint32_t* __restrict__ idx, uint64_t S, const uint32_t* __restrict__ e2, uint64_t n2,
    const uint32_t* __restrict__ g2_off, const uint32_t* __restrict__ g2_adj, Set64 hs2, Set128 hs3, Set128 hs4,
    const uint32_t* __restrict__ bits, uint32_t W, const uint8_t* __restrict__ lut_g,
    unsigned long long* __restrict__ hist, unsigned long long* __restrict__ ps) {
  __shared__ uint8_t lut[2048];
  __shared__ unsigned long long h_lds[256];
  load_lut(lut, lut_g, 2048);
  h_lds[threadIdx.x] = 0;
  __syncthreads();
  for (uint64_t s = blockIdx.x; s < S; s += gridDim.x) {
    const uint64_t i = idx[s];
    if (i >= n2) continue;
    unsigned long long* h = ps ? ps + s * 256 : h_lds;
    const uint32_t u = e2[2 * i], w = e2[2 * i + 1];
    const uint32_t ub = g2_off[u], du = g2_off[u + 1] - ub;
    const uint32_t wb = g2_off[w], dw = g2_off[w + 1] - wb;
    const uint64_t nL = uint64_t(du) + dw;
    auto valid = [&](uint32_t p, uint32_t x) {
      return x != u && x != w && (p < du || !pair_bit(hs2, bits, W, u, x));
    };
    // both other nodes adjacent to e
    const uint64_t npairs = nL * (nL - 1) / 2;
    for (uint64_t t = threadIdx.x; t < npairs; t += kThreads) {
      uint32_t p, q;
      pair_from_index(t, nL, p, q);
      const uint32_t x = nodeL(g2_adj, ub, du, wb, p), y = nodeL(g2_adj, ub, du, wb, q);
      if (!valid(p, x) || !valid(q, y)) continue;
      j2_candidate(u, w, x, y, hs2, hs3, hs4, bits, W, lut, h);
    }
    // x adjacent to e, y adjacent to x only
    for (uint32_t p = 0; p < nL; ++p) {
      const uint32_t x = nodeL(g2_adj, ub, du, wb, p);
      if (!valid(p, x)) continue;
      const uint32_t xb = g2_off[x], xe = g2_off[x + 1];
      for (uint32_t yi = xb + threadIdx.x; yi < xe; yi += kThreads) {
        const uint32_t y = g2_adj[yi];
        if (y == u || y == w || pair_bit(hs2, bits, W, u, y) || pair_bit(hs2, bits, W, w, y)) continue;
        j2_candidate(u, w, x, y, hs2, hs3, hs4, bits, W, lut, h);
      }
    }
  }
  __syncthreads();
  flush(h_lds, hist + kRaw, 256);
}

// order 3, j = 3: the sampled 3-node hyperedge with its pairs
__global__ void __launch_bounds__(kThreads) k_sample_j3_k3(const uint32_t* __restrict__ idx, uint64_t S,
                                                           const uint32_t* __restrict__ e3, uint64_t n3, Set64 hs2,
                                                           const uint32_t* __restrict__ bits, uint32_t W,
                                                           const uint8_t* __restrict__ lut_g,
                                                           unsigned long long* __restrict__ hist,
                                                           unsigned long long* __restrict__ ps) {
  __shared__ uint8_t lut[16];
  __shared__ unsigned long long h_lds[256];
  load_lut(lut, lut_g, 16);
  h_lds[threadIdx.x] = 0;
  __syncthreads();
  for (uint64_t s = uint64_t(blockIdx.x) * kThreads + threadIdx.x; s < S; s += uint64_t(gridDim.x) * kThreads) {
    const uint64_t i = idx[s];
    if (i >= n3) continue;
    unsigned long long* h = ps ? ps + s * 256 : h_lds;
    const uint32_t a = e3[3 * i], b = e3[3 * i + 1], c = e3[3 * i + 2];
    const uint32_t p = (1u << 3) | pair_bit(hs2, bits, W, a, b) | (pair_bit(hs2, bits, W, a, c) << 1) |
                       (pair_bit(hs2, bits, W, b, c) << 2);
    atomicAdd(&h[lut[p]], 1ull);
  }
  __syncthreads();
  flush(h_lds, hist + kRaw, 256);
}

// order 3, j = 2: the sampled pair {u, w} and one neighbour x of u or w
// (taken once) such that {u, w, x} is not a 3-node hyperedge.  One wavefront
// per sample.
__global__ void __launch_bounds__(kThreads) k_sample_j2_k3(const uint32_t* __restrict__ idx, uint64_t S,
                                                           const uint32_t* __restrict__ e2, uint64_t n2,
                                                           const uint32_t* __restrict__ g2_off,
                                                           const uint32_t* __restrict__ g2_adj, Set64 hs2,
                                                           Set128 hs3, const uint32_t* __restrict__ bits, uint32_t W,
                                                           const uint8_t* __restrict__ lut_g,
                                                           unsigned long long* __restrict__ hist,
                                                           unsigned long long* __restrict__ ps) {
  __shared__ uint8_t lut[16];
  __shared__ unsigned long long h_lds[256];
  load_lut(lut, lut_g, 16);
  h_lds[threadIdx.x] = 0;
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t wave = uint64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
  const uint64_t n_waves = uint64_t(gridDim.x) * kWavesPerBlock;
  for (uint64_t s = wave; s < S; s += n_waves) {
    const uint64_t i = idx[s];
    if (i >= n2) continue;
    const uint32_t u = e2[2 * i], w = e2[2 * i + 1];
    const uint32_t ub = g2_off[u], du = g2_off[u + 1] - ub;
    const uint32_t wb = g2_off[w], dw = g2_off[w + 1] - wb;
    unsigned long long* h = ps ? ps + s * 256 : h_lds;
    for (uint32_t p = lane; p < du + dw; p += kWave) {
      const uint32_t x = nodeL(g2_adj, ub, du, wb, p);
      if (x == u || x == w) continue;
      const uint32_t ux = pair_bit(hs2, bits, W, u, x);
      if (p >= du && ux) continue;            // taken from u's row
      uint32_t t0 = u, t1 = w, t2 = x;
      sort3(t0, t1, t2);
      if (set128_has(hs3, key3(t0, t1, t2))) continue;
      const uint32_t wx = pair_bit(hs2, bits, W, w, x);
      // local positions u=0, w=1, x=2
      atomicAdd(&h[lut[1u | (ux << 1) | (wx << 2)]], 1ull);
    }
  }
  __syncthreads();
  flush(h_lds, hist + kRaw, 256);
}

struct ScaleArgs {
  double n_by_size[5];
  double s_by_size[5];
  uint8_t maxcard[256];
  uint8_t countmax[256];
};

// est_m = raw_m * |E_mc| / (S_mc * countmax_m) in fp64, rounded once to fp32;
// 0 when the stratum was not sampled
__global__ void k_scale(const unsigned long long* __restrict__ hist, int n_classes, ScaleArgs args,
                        float* __restrict__ est, int64_t* __restrict__ raw) {
  const int c = threadIdx.x;
  if (c >= n_classes) return;
  const unsigned long long r = hist[kRaw + c];
  const int j = args.maxcard[c];
  double e = 0.0;
  if (args.s_by_size[j] > 0.0) e = (double(r) * args.n_by_size[j]) / (args.s_by_size[j] * double(args.countmax[c]));
  est[c] = float(e);
  if (raw) raw[c] = int64_t(r);
}

unsigned grid_for(uint64_t items, uint64_t per_block, unsigned cap = 512) {
  uint64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return unsigned(g);
}

int ensure_index_capacity(hm_graph* H, uint64_t n) {
  if (n <= H->sample_cap) return HM_OK;
  if (H->sample_idx) {
    HM_HIP(hipDeviceSynchronize());
    dfree(H->sample_idx);
    H->sample_idx = nullptr;
    H->sample_cap = 0;
  }
  void* p = nullptr;
  HM_TRY(dalloc(&p, n * sizeof(uint32_t)));
  H->sample_idx = static_cast<uint32_t*>(p);
  H->sample_cap = n;
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

// Enumerate around explicit samples (device index arrays).  With ps == null
// the raw counts go to hm_graph::hist; otherwise sample s of stratum j adds
// to row ps[row0[j] + s] (256 counters per row, zeroed by the caller).
int enumerate_samples(const hm_graph* H, int k, const uint32_t* const idx[5], const uint64_t S[5],
                      unsigned long long* ps, const uint64_t row0[5], hipStream_t st) {
  const uint8_t *lut4 = nullptr, *lut3 = nullptr;
  HM_TRY(device_luts(H->device, &lut4, &lut3));
  const uint64_t n2 = H->n_by_size[2], n3 = H->n_by_size[3], n4 = H->n_by_size[4];
  auto rows = [&](int j) { return ps ? ps + row0[j] * 256 : nullptr; };
  if (k == 4) {
    if (S[4]) {
      ProfileScope pscope("k_sample_j4", st);
      k_sample_j4<<<grid_for(S[4], kThreads), kThreads, 0, st>>>(idx[4], S[4], H->e4, n4, H->hs2, H->hs3, H->bits,
                                                                  H->words, lut4, H->hist, rows(4));
    }
    if (S[3]) {
      if (H->bits) {
        ProfileScope pscope("k_sample_j3_bits", st);
        k_sample_j3_bits<<<grid_for(S[3], kWavesPerBlock), kThreads, 0, st>>>(
            idx[3], S[3], H->e3, n3, H->e4, H->i3_off, H->i3_idx, H->i4_off, H->i4_idx, H->bits, H->words, lut4,
            H->hist, rows(3));
      } else {
        ProfileScope pscope("k_sample_j3_hash", st);
        k_sample_j3_hash<<<grid_for(S[3], kWavesPerBlock), kThreads, 0, st>>>(
            idx[3], S[3], H->e3, n3, H->g2_off, H->g2_adj, H->i3_off, H->i3_idx, H->hs2, H->hs3, H->hs4, lut4,
            H->hist, rows(3));
      }
    }
    if (S[2]) {
      ProfileScope pscope("k_sample_j2_k4", st);
      k_sample_j2_k4<<<grid_for(S[2], 1, 1024), kThreads, 0, st>>>(idx[2], S[2], H->e2, n2, H->g2_off, H->g2_adj,
                                                                    H->hs2, H->hs3, H->hs4, H->bits, H->words, lut4,
                                                                    H->hist, rows(2));
    }
  } else {
    if (S[3]) {
      ProfileScope pscope("k_sample_j3_k3", st);
      k_sample_j3_k3<<<grid_for(S[3], kThreads), kThreads, 0, st>>>(idx[3], S[3], H->e3, n3, H->hs2, H->bits,
                                                                     H->words, lut3, H->hist, rows(3));
    }
    if (S[2]) {
      ProfileScope pscope("k_sample_j2_k3", st);
      k_sample_j2_k3<<<grid_for(S[2], kWavesPerBlock), kThreads, 0, st>>>(idx[2], S[2], H->e2, n2, H->g2_off,
                                                                          H->g2_adj, H->hs2, H->hs3, H->bits,
                                                                          H->words, lut3, H->hist, rows(2));
    }
  }
  HM_HIP(hipGetLastError());
  return HM_OK;
}

// Enumerate around explicit samples and scale (Algorithm 4).
int sampled_from_indices(const hm_graph* H, int k, const uint32_t* const idx[5], const uint64_t S[5], float* est,
                         int64_t* raw, hipStream_t st) {
  HM_TRY(fill_u64(H->hist, 0, 4 * 256, st));
  const uint64_t row0[5] = {0, 0, 0, 0, 0};
  HM_TRY(enumerate_samples(H, k, idx, S, nullptr, row0, st));
  const ClassTables& t = class_tables();
  ScaleArgs a;
  for (int j = 0; j < 5; ++j) {
    a.n_by_size[j] = (j >= 2 && j <= 4) ? double(H->n_by_size[j]) : 0.0;
    a.s_by_size[j] = (j >= 2 && j <= k) ? double(S[j]) : 0.0;
  }
  for (int c = 0; c < 256; ++c) {
    a.maxcard[c] = c < t.n_classes[k] ? t.maxcard[k][c] : 0;
    a.countmax[c] = c < t.n_classes[k] ? t.countmax[k][c] : 1;
  }
  k_scale<<<1, 256, 0, st>>>(H->hist, t.n_classes[k], a, est, raw);
  HM_HIP(hipGetLastError());
  return HM_OK;
}

int draw_samples(hm_graph* H, int k, double fraction, uint64_t seed, int allocation, uint64_t S[5],
                 const uint32_t* idx[5], hipStream_t st) {
  HM_TRY(sample_sizes(H, k, fraction, allocation, S));
  const uint64_t total = S[2] + S[3] + S[4];
  HM_TRY(ensure_index_capacity(H, total + 1));
  uint64_t off = 0;
  for (int j = 0; j < 5; ++j) idx[j] = nullptr;
  for (int j = 2; j <= k; ++j) {
    idx[j] = H->sample_idx + off;
    if (S[j]) {
      k_draw<<<grid_for(S[j], 256, 1024), 256, 0, st>>>(H->sample_idx + off, S[j], H->n_by_size[j], seed,
                                                         uint32_t(j));
      HM_HIP(hipGetLastError());
    }
    off += S[j];
  }
  return HM_OK;
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
  const uint32_t* idx[5];
  HM_TRY(hm::draw_samples(const_cast<hm_graph*>(H), k, fraction, seed, allocation, S, idx, st));
  return hm::sampled_from_indices(H, k, idx, S, est, raw, st);
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
