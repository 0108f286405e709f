// Device primitives used while building graphs: exclusive scans, a stable
// LSD radix sort of (64-bit key, 32-bit value) pairs and fills.
#include <algorithm>

#include "hm_device.h"

namespace hm {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

template <typename T>
__device__ T block_exclusive_scan(T v, T* wave_sums, T* total) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const T x = wave_inclusive_scan(v);
  if (lane == kWave - 1) wave_sums[wave] = x;
  __syncthreads();
  T before = 0, all = 0;
  for (int w = 0; w < kScanThreads / kWave; ++w) {
    T s = wave_sums[w];
    if (w < wave) before += s;
    all += s;
  }
  __syncthreads();
  *total = all;
  return before + x - v;
}

template <typename T>
__global__ void __launch_bounds__(kScanThreads) k_scan_tile(const T* __restrict__ in, T* __restrict__ out,
                                                            T* __restrict__ sums, uint64_t n) {
  __shared__ T tile[kScanTile];
  __shared__ T wave_sums[kScanThreads / kWave];
  const uint64_t base = uint64_t(blockIdx.x) * kScanTile;
  // (all of the thread's loads before its LDS stores, so that they go out
  // together)
  T v[kScanItems];
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const uint64_t g = base + uint64_t(r) * kScanThreads + threadIdx.x;
    v[r] = g < n ? in[g] : T(0);
  }
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) tile[r * kScanThreads + threadIdx.x] = v[r];
  __syncthreads();
  T local[kScanItems];
  T s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    local[j] = tile[threadIdx.x * kScanItems + j];
    s += local[j];
  }
  T total;
  T off = block_exclusive_scan(s, wave_sums, &total);
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    tile[threadIdx.x * kScanItems + j] = off;
    off += local[j];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kScanTile; i += kScanThreads) {
    uint64_t g = base + i;
    if (g < n) out[g] = tile[i];
  }
  if (threadIdx.x == 0 && sums) sums[blockIdx.x] = total;
}

template <typename T>
__global__ void k_scan_add(T* __restrict__ out, const T* __restrict__ offs, uint64_t n) {
  uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] += offs[i / kScanTile];
}

template <typename T>
__global__ void k_scan_total(const T* in, const T* out, uint64_t n, T* total) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *total = n ? out[n - 1] + in[n - 1] : T(0);
}

template <typename T>
int scan_impl(const T* in, T* out, uint64_t n, hipStream_t st) {
  if (n == 0) return HM_OK;
  const uint64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 1) {
    k_scan_tile<T><<<1, kScanThreads, 0, st>>>(in, out, nullptr, n);
    HM_HIP(hipGetLastError());
    return HM_OK;
  }
  void* sums = nullptr;
  void* sums_scan = nullptr;
  HM_TRY(dalloc(&sums, nb * sizeof(T)));
  int rc = dalloc(&sums_scan, nb * sizeof(T));
  if (rc != HM_OK) {
    dfree(sums);
    return rc;
  }
  k_scan_tile<T><<<unsigned(nb), kScanThreads, 0, st>>>(in, out, static_cast<T*>(sums), n);
  rc = (hipGetLastError() == hipSuccess) ? HM_OK : HM_EDEVICE;
  if (rc == HM_OK) rc = scan_impl<T>(static_cast<T*>(sums), static_cast<T*>(sums_scan), nb, st);
  if (rc == HM_OK) {
    k_scan_add<T><<<unsigned((n + 255) / 256), 256, 0, st>>>(out, static_cast<T*>(sums_scan), n);
    rc = (hipGetLastError() == hipSuccess) ? HM_OK : HM_EDEVICE;
  }
  (void)hipStreamSynchronize(st);
  dfree(sums);
  dfree(sums_scan);
  if (rc == HM_EDEVICE) set_error("scan kernel launch failed");
  return rc;
}

// ------------------------------------------------------------------ radix sort
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kSortWaves = kSortThreads / kWave;

__global__ void __launch_bounds__(kSortThreads) k_sort_hist(const unsigned long long* __restrict__ keys,
                                                            uint64_t n, int shift, uint32_t digit_mask,
                                                            uint32_t* __restrict__ hist, uint32_t nb) {
  __shared__ uint32_t counts[256];
  counts[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t base = uint64_t(blockIdx.x) * kSortTile;
  // every key of the thread loaded before any is counted (the loads go out
  // together rather than each behind the previous count)
  uint32_t d[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const uint64_t i = base + uint64_t(r) * kSortThreads + threadIdx.x;
    d[r] = i < n ? uint32_t(keys[i] >> shift) & digit_mask : 0xFFFFFFFFu;
  }
#pragma unroll
  for (int r = 0; r < kSortItems; ++r)
    if (d[r] != 0xFFFFFFFFu) atomicAdd(&counts[d[r]], 1u);
  __syncthreads();
  hist[uint64_t(threadIdx.x) * nb + blockIdx.x] = counts[threadIdx.x];
}

// Stable scatter in two steps.  First the tile is sorted by digit in LDS:
// items are taken round by round (position order is round-major, then
// thread), ranks inside a wavefront come from ballots over the digit bits and
// ranks across wavefronts from per-round LDS counts, on top of the tile's own
// digit offsets (the exclusive scan of its counts from k_sort_hist).  Then
// thread t writes the tile's t-th item in digit order to its digit's global
// range, so that each digit's items of the tile go out as one contiguous run.
__global__ void __launch_bounds__(kSortThreads) k_sort_scatter(
    const unsigned long long* __restrict__ keys, const uint32_t* __restrict__ vals,
    unsigned long long* __restrict__ out_keys, uint32_t* __restrict__ out_vals, uint64_t n, int shift,
    int digit_bits, const uint32_t* __restrict__ hist, const uint32_t* __restrict__ offsets, uint32_t nb) {
  __shared__ unsigned long long s_keys[kSortTile];
  __shared__ uint32_t s_vals[kSortTile];
  __shared__ uint32_t tile_off[256], global_off[256], running[256];
  __shared__ uint32_t wave_cnt[kSortWaves][256];
  __shared__ uint32_t wave_sums[kSortWaves];
  const uint32_t digit_mask = (1u << digit_bits) - 1u;
  {
    const uint32_t c = hist[uint64_t(threadIdx.x) * nb + blockIdx.x];
    uint32_t total;
    const uint32_t off = block_exclusive_scan(c, wave_sums, &total);
    tile_off[threadIdx.x] = off;
    running[threadIdx.x] = off;
    global_off[threadIdx.x] = offsets[uint64_t(threadIdx.x) * nb + blockIdx.x];
  }
  for (int w = 0; w < kSortWaves; ++w) wave_cnt[w][threadIdx.x] = 0;
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const unsigned long long lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  const uint64_t base = uint64_t(blockIdx.x) * kSortTile;
  // the tile's items, all loads issued before the first is needed
  unsigned long long rk[kSortItems];
  uint32_t rv[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const uint64_t i = base + uint64_t(r) * kSortThreads + threadIdx.x;
    rk[r] = i < n ? keys[i] : 0ull;
    rv[r] = i < n ? vals[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const uint64_t i = base + uint64_t(r) * kSortThreads + threadIdx.x;
    const bool valid = i < n;
    const unsigned long long key = rk[r];
    const uint32_t val = rv[r];
    const uint32_t d = valid ? uint32_t(key >> shift) & digit_mask : 0u;
    unsigned long long peers = __ballot(valid);
    for (int b = 0; b < digit_bits; ++b) {
      const bool bit = (d >> b) & 1u;
      const unsigned long long bal = __ballot(valid && bit);
      peers &= bit ? bal : ~bal;
    }
    const uint32_t rank = __popcll(peers & lt_mask);
    if (valid && rank == 0) wave_cnt[wave][d] = uint32_t(__popcll(peers));
    __syncthreads();
    if (valid) {
      uint32_t pos = running[d] + rank;
      for (int w = 0; w < wave; ++w) pos += wave_cnt[w][d];
      s_keys[pos] = key;
      s_vals[pos] = val;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < kSortWaves; ++w) {
      add += wave_cnt[w][threadIdx.x];
      wave_cnt[w][threadIdx.x] = 0;
    }
    running[threadIdx.x] += add;
    __syncthreads();
  }
  const uint32_t tile_n = uint32_t(min<uint64_t>(uint64_t(kSortTile), n - base));
  for (uint32_t j = threadIdx.x; j < tile_n; j += kSortThreads) {
    const unsigned long long key = s_keys[j];
    const uint32_t d = uint32_t(key >> shift) & digit_mask;
    const uint32_t pos = global_off[d] + (j - tile_off[d]);
    out_keys[pos] = key;
    out_vals[pos] = s_vals[j];
  }
}

template <typename T>
__global__ void k_fill(T* p, T value, uint64_t n) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
    p[i] = value;
}

template <typename T>
int fill_impl(T* p, T value, uint64_t n, hipStream_t st) {
  if (n == 0) return HM_OK;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  k_fill<T><<<unsigned(blocks), 256, 0, st>>>(p, value, n);
  HM_HIP(hipGetLastError());
  return HM_OK;
}

template <typename T>
__global__ void k_copy(const T* __restrict__ src, T* __restrict__ dst, uint64_t n) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
    dst[i] = src[i];
}

}  // namespace

// ------------------------------------------------------------------ planned (workspace) variants
// Multi-level exclusive scan of up to n uint32 values: level l scans the
// block sums of level l-1.  No allocation and no host synchronisation.
uint64_t scan_ws_words(uint64_t n) {
  uint64_t words = 0;
  while (n > uint64_t(kScanTile)) {
    n = (n + kScanTile - 1) / kScanTile;
    words += 2 * n;    // block sums and their scan
  }
  return words + 1;
}

int scan_u32_ws(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* total_dev, uint32_t* ws, hipStream_t st) {
  if (n == 0) {
    if (total_dev) HM_TRY(fill_u32(total_dev, 0, 1, st));
    return HM_OK;
  }
  const uint64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 1) {
    k_scan_tile<uint32_t><<<1, kScanThreads, 0, st>>>(in, out, nullptr, n);
  } else {
    uint32_t* sums = ws;
    uint32_t* sums_scan = ws + nb;
    k_scan_tile<uint32_t><<<unsigned(nb), kScanThreads, 0, st>>>(in, out, sums, n);
    HM_HIP(hipGetLastError());
    HM_TRY(scan_u32_ws(sums, sums_scan, nb, nullptr, ws + 2 * nb, st));
    k_scan_add<uint32_t><<<unsigned((n + 255) / 256), 256, 0, st>>>(out, sums_scan, n);
  }
  HM_HIP(hipGetLastError());
  if (total_dev) {
    k_scan_total<uint32_t><<<1, 1, 0, st>>>(in, out, n, total_dev);
    HM_HIP(hipGetLastError());
  }
  return HM_OK;
}

uint64_t radix_ws_words(uint64_t n) {
  const uint64_t nb = (n + kSortTile - 1) / kSortTile;
  return 2 * 256 * nb + scan_ws_words(256 * nb) + 16;
}

int radix_sort_ws(unsigned long long* keys, uint32_t* vals, unsigned long long* keys_tmp, uint32_t* vals_tmp,
                  uint64_t n, int bits, uint32_t* ws, hipStream_t st) {
  if (n <= 1 || bits <= 0) return HM_OK;
  if (bits > 64) bits = 64;
  const uint64_t nb64 = (n + kSortTile - 1) / kSortTile;
  if (nb64 > 0xFFFFFFull) {
    set_error("radix sort of %llu items is too large", (unsigned long long)n);
    return HM_EUNSUPPORTED;
  }
  const uint32_t nb = uint32_t(nb64);
  uint32_t* hist = ws;
  uint32_t* offs = ws + size_t(256) * nb;
  uint32_t* scan_ws = ws + size_t(512) * nb;
  unsigned long long* src_k = keys;
  uint32_t* src_v = vals;
  unsigned long long* dst_k = keys_tmp;
  uint32_t* dst_v = vals_tmp;
  for (int shift = 0; shift < bits; shift += 8) {
    const int db = (bits - shift) < 8 ? (bits - shift) : 8;
    k_sort_hist<<<nb, kSortThreads, 0, st>>>(src_k, n, shift, (1u << db) - 1u, hist, nb);
    HM_HIP(hipGetLastError());
    HM_TRY(scan_u32_ws(hist, offs, uint64_t(256) * nb, nullptr, scan_ws, st));
    k_sort_scatter<<<nb, kSortThreads, 0, st>>>(src_k, src_v, dst_k, dst_v, n, shift, db, hist, offs, nb);
    HM_HIP(hipGetLastError());
    std::swap(src_k, dst_k);
    std::swap(src_v, dst_v);
  }
  if (src_k != keys) {
    const unsigned g = unsigned(std::min<uint64_t>((n + 255) / 256, 16384));
    k_copy<unsigned long long><<<g, 256, 0, st>>>(src_k, keys, n);
    k_copy<uint32_t><<<g, 256, 0, st>>>(src_v, vals, n);
    HM_HIP(hipGetLastError());
  }
  return HM_OK;
}

int copy_u32(const uint32_t* src, uint32_t* dst, uint64_t n, hipStream_t st) {
  if (!n) return HM_OK;
  k_copy<uint32_t><<<unsigned(std::min<uint64_t>((n + 255) / 256, 16384)), 256, 0, st>>>(src, dst, n);
  HM_HIP(hipGetLastError());
  return HM_OK;
}

int copy_u64(const unsigned long long* src, unsigned long long* dst, uint64_t n, hipStream_t st) {
  if (!n) return HM_OK;
  k_copy<unsigned long long><<<unsigned(std::min<uint64_t>((n + 255) / 256, 16384)), 256, 0, st>>>(src, dst, n);
  HM_HIP(hipGetLastError());
  return HM_OK;
}

int scan_exclusive_u32(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* total_dev, hipStream_t st) {
  HM_TRY(scan_impl<uint32_t>(in, out, n, st));
  if (total_dev) {
    k_scan_total<uint32_t><<<1, 1, 0, st>>>(in, out, n, total_dev);
    HM_HIP(hipGetLastError());
  }
  return HM_OK;
}

int scan_exclusive_u64(const unsigned long long* in, unsigned long long* out, uint64_t n, hipStream_t st) {
  return scan_impl<unsigned long long>(in, out, n, st);
}

int radix_sort_pairs(unsigned long long* keys, uint32_t* vals, unsigned long long* keys_tmp, uint32_t* vals_tmp,
                     uint64_t n, int bits, hipStream_t st) {
  if (n <= 1 || bits <= 0) return HM_OK;
  if (bits > 64) bits = 64;
  const uint64_t nb64 = (n + kSortTile - 1) / kSortTile;
  if (nb64 > 0xFFFFFFull) {
    set_error("radix sort of %llu items is too large", (unsigned long long)n);
    return HM_EUNSUPPORTED;
  }
  const uint32_t nb = uint32_t(nb64);
  void* hist = nullptr;
  void* offs = nullptr;
  HM_TRY(dalloc(&hist, size_t(256) * nb * sizeof(uint32_t)));
  int rc = dalloc(&offs, size_t(256) * nb * sizeof(uint32_t));
  if (rc != HM_OK) {
    dfree(hist);
    return rc;
  }
  unsigned long long* src_k = keys;
  uint32_t* src_v = vals;
  unsigned long long* dst_k = keys_tmp;
  uint32_t* dst_v = vals_tmp;
  for (int shift = 0; shift < bits && rc == HM_OK; shift += 8) {
    const int db = (bits - shift) < 8 ? (bits - shift) : 8;
    const uint32_t mask = (1u << db) - 1u;
    k_sort_hist<<<nb, kSortThreads, 0, st>>>(src_k, n, shift, mask, static_cast<uint32_t*>(hist), nb);
    if (hipGetLastError() != hipSuccess) rc = HM_EDEVICE;
    if (rc == HM_OK)
      rc = scan_exclusive_u32(static_cast<uint32_t*>(hist), static_cast<uint32_t*>(offs), uint64_t(256) * nb,
                              nullptr, st);
    if (rc == HM_OK) {
      k_sort_scatter<<<nb, kSortThreads, 0, st>>>(src_k, src_v, dst_k, dst_v, n, shift, db,
                                                  static_cast<const uint32_t*>(hist), static_cast<uint32_t*>(offs), nb);
      if (hipGetLastError() != hipSuccess) rc = HM_EDEVICE;
    }
    std::swap(src_k, dst_k);
    std::swap(src_v, dst_v);
  }
  if (rc == HM_OK && src_k != keys) {
    if (hipMemcpyAsync(keys, src_k, n * sizeof(unsigned long long), hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(vals, src_v, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st) != hipSuccess)
      rc = HM_EDEVICE;
  }
  (void)hipStreamSynchronize(st);
  dfree(hist);
  dfree(offs);
  if (rc == HM_EDEVICE) set_error("radix sort kernel failed");
  return rc;
}

int fill_u32(uint32_t* p, uint32_t value, uint64_t n, hipStream_t st) { return fill_impl<uint32_t>(p, value, n, st); }

int fill_u64(unsigned long long* p, unsigned long long value, uint64_t n, hipStream_t st) {
  return fill_impl<unsigned long long>(p, value, n, st);
}

__global__ void k_max_u32(const uint32_t* __restrict__ v, uint64_t n, uint32_t* out) {
  uint32_t m = 0;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
    m = v[i] > m ? v[i] : m;
  for (int d = kWave / 2; d > 0; d >>= 1) {
    const uint32_t o = __shfl_xor(m, d, kWave);
    m = o > m ? o : m;
  }
  if ((threadIdx.x & (kWave - 1)) == 0 && m) atomicMax(out, m);
}

int max_u32(const uint32_t* v, uint64_t n, uint32_t* out, hipStream_t st) {
  if (!n) return HM_OK;
  uint64_t g = (n + 255) / 256;
  if (g > 1024) g = 1024;
  k_max_u32<<<unsigned(g), 256, 0, st>>>(v, n, out);
  HM_HIP(hipGetLastError());
  return HM_OK;
}

}  // namespace hm
