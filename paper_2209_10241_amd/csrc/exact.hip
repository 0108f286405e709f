// Exact counting of order-3 and order-4 higher-order motifs (Algorithms 2
// and 3, Section 4.2) on gfx950.
//
// Algorithm 3 finds every connected 4-node set once by three generators and a
// global "visited" set of node sets; here the visited set is replaced by
// ownership rules decided from the node set alone (hm_items.h, hm_b4.h), so
// every generator instance runs independently.  Every counted set is
// classified by fill-in (existence of each sub-hyperedge, Section 4.3
// Fig. 3b) and one read of the pattern->class table (Section 4.3 Fig. 3a)
// held in LDS; per-class counters live in LDS and are flushed to device
// memory with one atomic per class per workgroup.
#include <vector>

#include "hm_items.h"

namespace hm {
namespace {

// (a) at order 4: one thread per 4-node hyperedge.
__global__ void __launch_bounds__(kThreads) k_case_a4(View v, uint64_t n4, const uint8_t* __restrict__ lut_g,
                                                      unsigned long long* __restrict__ hist) {
  __shared__ uint8_t lut[2048];
  __shared__ unsigned long long h_main[256], h_sub[256];
  load_lut(lut, lut_g, 2048);
  h_main[threadIdx.x] = 0;
  h_sub[threadIdx.x] = 0;
  __syncthreads();
  for (uint64_t i = uint64_t(blockIdx.x) * kThreads + threadIdx.x; i < n4; i += uint64_t(gridDim.x) * kThreads) {
    const uint32_t p = a4_pattern(v, v.e4[4 * i], v.e4[4 * i + 1], v.e4[4 * i + 2], v.e4[4 * i + 3]);
    count_class(lut, h_main, h_sub, p, kPairBits4);
  }
  __syncthreads();
  flush(h_main, hist + kMain, 256);
  flush(h_sub, hist + kSub, 256);
}

// (b) at order 4: one wavefront per 3-node hyperedge.
__global__ void __launch_bounds__(kThreads) k_case_b4(View v, uint64_t n3, const uint8_t* __restrict__ lut_g,
                                                      unsigned long long* __restrict__ hist) {
  __shared__ uint8_t lut[2048];
  __shared__ unsigned long long h_main[256], h_sub[256];
  __shared__ B4Scratch scratch[kWavesPerBlock];
  load_lut(lut, lut_g, 2048);
  h_main[threadIdx.x] = 0;
  h_sub[threadIdx.x] = 0;
  __syncthreads();
  const int wv = threadIdx.x / kWave;
  const uint64_t wave = uint64_t(blockIdx.x) * kWavesPerBlock + wv;
  const uint64_t n_waves = uint64_t(gridDim.x) * kWavesPerBlock;
  for (uint64_t i = wave; i < n3; i += n_waves) b4_item(v, i, &scratch[wv], lut, h_main, h_sub);
  __syncthreads();
  flush(h_main, hist + kMain, 256);
  flush(h_sub, hist + kSub, 256);
}

// (c) at order 4: one wavefront per pair {r < x} of G2.
__global__ void __launch_bounds__(kThreads) k_case_c4_bits(View v, uint64_t n2, const uint8_t* __restrict__ lut_g,
                                                           unsigned long long* __restrict__ hist) {
  __shared__ uint8_t lut[2048];
  __shared__ unsigned long long h_g2[256];
  __shared__ uint32_t ylist[kWavesPerBlock][kWave];
  load_lut(lut, lut_g, 2048);
  h_g2[threadIdx.x] = 0;
  __syncthreads();
  const int wv = threadIdx.x / kWave;
  const uint64_t wave = uint64_t(blockIdx.x) * kWavesPerBlock + wv;
  const uint64_t n_waves = uint64_t(gridDim.x) * kWavesPerBlock;
  const C4Lanes L = c4_lanes(v.W);
  C4Acc acc;
  c4_zero(acc);
  for (uint64_t i = wave; i < n2; i += n_waves) c4_bits_item(v, v.e2[2 * i], v.e2[2 * i + 1], L, ylist[wv], acc);
  c4_flush(acc, lut, h_g2);
  __syncthreads();
  flush(h_g2, hist + kG2, 256);
}

// (a) at order 3: one thread per 3-node hyperedge.
__global__ void __launch_bounds__(kThreads) k_case_a3(View v, uint64_t n3, const uint8_t* __restrict__ lut_g,
                                                      unsigned long long* __restrict__ hist) {
  __shared__ uint8_t lut[16];
  __shared__ unsigned long long h_main[256], h_sub[256];
  load_lut(lut, lut_g, 16);
  h_main[threadIdx.x] = 0;
  h_sub[threadIdx.x] = 0;
  __syncthreads();
  for (uint64_t i = uint64_t(blockIdx.x) * kThreads + threadIdx.x; i < n3; i += uint64_t(gridDim.x) * kThreads)
    count_class(lut, h_main, h_sub, a3_pattern(v, v.e3[3 * i], v.e3[3 * i + 1], v.e3[3 * i + 2]), kPairBits3);
  __syncthreads();
  flush(h_main, hist + kMain, 256);
  flush(h_sub, hist + kSub, 256);
}

// (c) at order 3 with bit rows: one thread per (pair, word).
__global__ void __launch_bounds__(kThreads) k_case_c3_bits(View v, uint64_t n2, const uint8_t* __restrict__ lut_g,
                                                           unsigned long long* __restrict__ hist) {
  __shared__ uint8_t lut[16];
  __shared__ unsigned long long h_g2[256];
  load_lut(lut, lut_g, 16);
  h_g2[threadIdx.x] = 0;
  __syncthreads();
  C3Acc acc{0, 0, 0};
  const uint64_t tasks = n2 * v.W;
  for (uint64_t t = uint64_t(blockIdx.x) * kThreads + threadIdx.x; t < tasks; t += uint64_t(gridDim.x) * kThreads) {
    const uint64_t i = t / v.W;
    c3_bits_word(v, v.e2[2 * i], v.e2[2 * i + 1], uint32_t(t % v.W), acc);
  }
  c3_flush(acc, lut, h_g2);
  __syncthreads();
  flush(h_g2, hist + kG2, 256);
}

// counts[c] = main[c] + (c pairs-only ? g2[c] - sub[c] : 0), as int64
struct ClassMask {
  unsigned long long w[4];
};

__global__ void k_combine(const unsigned long long* __restrict__ hist, int n_classes, ClassMask pairs_only,
                          int64_t* __restrict__ counts) {
  const int c = threadIdx.x;
  if (c >= n_classes) return;
  unsigned long long v = hist[kMain + c];
  if ((pairs_only.w[c >> 6] >> (c & 63)) & 1ull) v += hist[kG2 + c] - hist[kSub + c];
  counts[c] = int64_t(v);
}

// Counting kernels keep per-class counters in LDS and flush them once per
// workgroup; a grid of a few workgroups per CU that strides over the work
// keeps those flushes (global atomics on a few hundred addresses) rare.
constexpr unsigned kCountGrid = 512;

unsigned grid_waves(uint64_t items, unsigned cap = kCountGrid) {
  uint64_t g = (items + kWavesPerBlock - 1) / kWavesPerBlock;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return unsigned(g);
}
unsigned grid_threads(uint64_t items, unsigned cap = kCountGrid, unsigned per_block = kThreads) {
  uint64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return unsigned(g);
}

}  // namespace

int count_exact_impl(const hm_graph* H, int k, int64_t* counts, hipStream_t st) {
  const uint8_t *lut4 = nullptr, *lut3 = nullptr;
  HM_TRY(device_luts(H->device, &lut4, &lut3));
  const ClassTables& t = class_tables();
  ClassMask pairs_only{{0, 0, 0, 0}};
  for (int c = 0; c < t.n_classes[k]; ++c)
    if (t.maxcard[k][c] == 2) pairs_only.w[c >> 6] |= 1ull << (c & 63);
  HM_TRY(fill_u64(H->hist, 0, 4 * 256, st));
  const uint64_t n2 = H->n_by_size[2], n3 = H->n_by_size[3], n4 = H->n_by_size[4];
  const View v = view_of(H);
  if (k == 4) {
    if (n4) {
      ProfileScope ps("k_case_a4", st);
      k_case_a4<<<grid_threads(n4), kThreads, 0, st>>>(v, n4, lut4, H->hist);
    }
    if (v.bits) {
      if (n3) {
        ProfileScope ps("k_case_b4_bits", st);
        k_case_b4<<<grid_waves(n3), kThreads, 0, st>>>(v, n3, lut4, H->hist);
      }
      if (n2) {
        ProfileScope ps("k_case_c4_bits", st);
        k_case_c4_bits<<<grid_waves(n2), kThreads, 0, st>>>(v, n2, lut4, H->hist);
      }
    }
  } else {
    if (n3) {
      ProfileScope ps("k_case_a3", st);
      k_case_a3<<<grid_threads(n3), kThreads, 0, st>>>(v, n3, lut3, H->hist);
    }
    if (v.bits && n2) {
      ProfileScope ps("k_case_c3_bits", st);
      k_case_c3_bits<<<grid_threads(n2 * v.W), kThreads, 0, st>>>(v, n2, lut3, H->hist);
    }
  }
  HM_HIP(hipGetLastError());
  if (!v.bits) HM_TRY(count_sparse(H, k, st));
  HM_HIP(hipGetLastError());
  k_combine<<<1, 256, 0, st>>>(H->hist, t.n_classes[k], pairs_only, counts);
  HM_HIP(hipGetLastError());
  return HM_OK;
}

}  // namespace hm

extern "C" int count_exact(const hm_graph* H, int k, int64_t* counts, void* stream) {
  if (!H || !counts) {
    hm::set_error("NULL argument to count_exact");
    return HM_EINVAL;
  }
  if (k != 3 && k != 4) {
    hm::set_error("order %d is not supported (3 or 4)", k);
    return HM_EUNSUPPORTED;
  }
  return hm::count_exact_impl(H, k, counts, static_cast<hipStream_t>(stream));
}
