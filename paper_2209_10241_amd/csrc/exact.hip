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
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
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
  unsigned long long* hc = hist_copy(hist, kExactHistStride);
  flush(h_main, hc + kMain, 256);
  flush(h_sub, hc + kSub, 256);
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
  unsigned long long* hc = hist_copy(hist, kExactHistStride);
  flush(h_main, hc + kMain, 256);
  flush(h_sub, hc + kSub, 256);
}

// counts[c] = main[c] + (c pairs-only ? g2[c] - sub[c] : 0), as int64
struct ClassMask {
  unsigned long long w[4];
};

// (one workgroup of 256 threads; sums the kHistCopies copies of hist and
// leaves them zero)
__global__ void __launch_bounds__(256) k_combine(unsigned long long* __restrict__ hist, int n_classes, ClassMask pairs_only,
                          int64_t* __restrict__ counts, IdShapes sh) {
  __shared__ unsigned long long ids[8];
  const int c = threadIdx.x;
  // every copy is read before any is cleared, so that the loads go out
  // together rather than each behind the previous store
  // (all 4 x kHistCopies loads are issued before any is summed; the
  // identity sums are read by every thread, inside the copy's stride, and
  // kept by the first seven, since a conditional load would wait for the
  // loads before it)
  const bool ids_on = sh.on && c < 7;
  unsigned long long lm[kHistCopies], ls[kHistCopies], lg[kHistCopies], la[kHistCopies];
#pragma unroll
  for (uint32_t q = 0; q < kHistCopies; ++q) {
    const unsigned long long* h = hist + uint64_t(q) * kExactHistStride;
    lm[q] = h[kMain + c];
    ls[q] = h[kSub + c];
    lg[q] = h[kG2 + c];
    la[q] = h[kIdAcc + c];
  }
  unsigned long long m = 0, s = 0, g = 0, a = 0;
#pragma unroll
  for (uint32_t q = 0; q < kHistCopies; ++q) {
    m += lm[q];
    s += ls[q];
    g += lg[q];
    a += ids_on ? la[q] : 0ull;
  }
  __syncthreads();
#pragma unroll
  for (uint32_t q = 0; q < kHistCopies; ++q) {
    unsigned long long* h = hist + uint64_t(q) * kExactHistStride;
    h[kMain + c] = 0;
    h[kSub + c] = 0;
    h[kG2 + c] = 0;
    if (sh.on && c < 7) h[kIdAcc + c] = 0;
  }
  if (sh.on) {
    if (c < 7) ids[c] = a;
    __syncthreads();
    g = id_shape_count(ids, sh, c);
  }
  if (c < n_classes) {
    unsigned long long v = m;
    if ((pairs_only.w[c >> 6] >> (c & 63)) & 1ull) v += g - s;
    counts[c] = int64_t(v);
  }
}

// All generators of one order in a single launch (bit rows), sized to the
// workgroups resident at once.  The work of the three cases is laid out as
// one list that every wavefront (order 4) or thread (order 3) strides over,
// so each takes a like share of every case and no case waits for another.
// The counters go to the main, sub and G2 regions of hist; k_combine forms
// the counts afterwards (a kernel boundary, rather than a device-wide fence
// in every workgroup, makes the atomics of all workgroups visible to it).
constexpr uint32_t kA4Chunk = kWave;   // 4-node hyperedges per wavefront item
// Largest bit matrix and row starts a workgroup copies into LDS (about 500
// nodes): several workgroups per CU still fit beside them.
constexpr size_t kLdsBitsMaxBytes = 40960;

// Workgroups of the order-4 launch: 16 wavefronts, so that the tables it
// copies into LDS are read once per CU and its counters flushed once per CU.
constexpr uint32_t kExact4Waves = 16;
constexpr uint32_t kExact4Threads = kExact4Waves * kWave;

struct ExactArgs {
  View v;
  uint64_t n2, n3, n4;
  const uint8_t* lut;
  unsigned long long* hist;
};

// Order 4: items [0, n2) are the pairs of G2 (case (c)), [n2, n2 + n3) the
// 3-node hyperedges (case (b)), then chunks of kA4Chunk 4-node hyperedges
// (case (a)).  Dynamic LDS holds b4_set_words(W) words per wavefront and,
// with LB, a copy of the whole bit matrix (N x W words) and of the row
// starts of G2 and of the incidence lists, so that every adjacency word and
// row bound the items read comes from LDS rather than from L2.
template <bool LB, bool ID>
__global__ void __launch_bounds__(kExact4Threads) k_exact4_bits(ExactArgs a) {
  __shared__ uint8_t lut[2048];
  __shared__ unsigned long long h_main[256], h_sub[256], h_g2[256], h_id[8];
  __shared__ uint32_t ylist[kExact4Waves][kWave];
  extern __shared__ uint32_t dyn_lds[];
  View v = a.v;
  uint32_t* b4_sets = dyn_lds;
  if (LB) {
    // the rows start 16 * (4 * W + 64) words in: 16-byte aligned
    uint32_t* rows = dyn_lds + kExact4Waves * b4_set_words(v.W);
    const uint32_t n = v.N * v.W, n4 = n / 4;
    const uint4* src = reinterpret_cast<const uint4*>(v.bits);
    uint4* dst = reinterpret_cast<uint4*>(rows);
    for (uint32_t i = threadIdx.x; i < n4; i += kExact4Threads) dst[i] = src[i];
    for (uint32_t i = 4 * n4 + threadIdx.x; i < n; i += kExact4Threads) rows[i] = v.bits[i];
    // and the row starts of G2 and of the incidence lists
    uint32_t* offs = rows + n;
    for (uint32_t i = threadIdx.x; i <= v.N; i += kExact4Threads) {
      offs[i] = v.g2_off[i];
      offs[v.N + 1 + i] = v.i3_off[i];
      offs[2 * (v.N + 1) + i] = v.i4_off[i];
    }
    v.bits = rows;
    v.g2_off = offs;
    v.i3_off = offs + v.N + 1;
    v.i4_off = offs + 2 * (v.N + 1);
  }
  load_lut(lut, a.lut, 2048);
  if (threadIdx.x < 256) {
    h_main[threadIdx.x] = 0;
    h_sub[threadIdx.x] = 0;
    h_g2[threadIdx.x] = 0;
  }
  if (threadIdx.x < 8) h_id[threadIdx.x] = 0;
  __syncthreads();
  const int wv = threadIdx.x / kWave;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  uint32_t* sets = b4_sets + wv * b4_set_words(v.W);
  const C4Lanes L = c4_lanes(v.W);
  C4Acc acc;
  IdAcc ida;
  if (ID) id_zero(ida); else c4_zero(acc);
  // (c) items: the pairs of G2, then (identity route) one per node
  const uint64_t nc = ID ? a.n2 + v.N : a.n2;
  const uint64_t n23 = nc + a.n3;
  const uint64_t items = n23 + (a.n4 + kA4Chunk - 1) / kA4Chunk;
  const uint64_t n_waves = uint64_t(gridDim.x) * kExact4Waves;
  for (uint64_t i = uint64_t(blockIdx.x) * kExact4Waves + wv; i < items; i += n_waves) {
    if (i < a.n2) {
      if (ID) id_edge_item(v, v.e2[2 * i], v.e2[2 * i + 1], L, ylist[wv], ida);
      else c4_bits_item(v, v.e2[2 * i], v.e2[2 * i + 1], L, ylist[wv], acc, lut, h_g2);
    } else if (i < nc) {
      id_node_item(v, uint32_t(i - a.n2), ida);
    } else if (i < n23) {
      b4_item(v, i - nc, sets, lut, h_main, h_sub);
    } else {
      const uint64_t e = (i - n23) * kA4Chunk + lane;
      if (e < a.n4)
        count_class(lut, h_main, h_sub, a4_pattern(v, v.e4[4 * e], v.e4[4 * e + 1], v.e4[4 * e + 2], v.e4[4 * e + 3]),
                    kPairBits4);
    }
  }
  if (ID) id_flush(ida, h_id); else c4_flush(acc, lut, h_g2);
  __syncthreads();
  unsigned long long* hc = hist_copy(a.hist, kExactHistStride);
  flush(h_main, hc + kMain, 256);
  flush(h_sub, hc + kSub, 256);
  if (ID) flush(h_id, hc + kIdAcc, 8); else flush(h_g2, hc + kG2, 256);
}

// Order 3: thread items [0, n2 * W) are the (pair, word) tasks of case (c),
// then one per 3-node hyperedge (case (a)).
__global__ void __launch_bounds__(kThreads) k_exact3_bits(ExactArgs a) {
  __shared__ uint8_t lut[16];
  __shared__ unsigned long long h_main[256], h_sub[256], h_g2[256];
  load_lut(lut, a.lut, 16);
  h_main[threadIdx.x] = 0;
  h_sub[threadIdx.x] = 0;
  h_g2[threadIdx.x] = 0;
  __syncthreads();
  const View& v = a.v;
  C3Acc acc{0, 0, 0};
  const uint64_t tasks = a.n2 * v.W;
  const uint64_t items = tasks + a.n3;
  for (uint64_t t = uint64_t(blockIdx.x) * kThreads + threadIdx.x; t < items; t += uint64_t(gridDim.x) * kThreads) {
    if (t < tasks) {
      const uint64_t i = t / v.W;
      c3_bits_word(v, v.e2[2 * i], v.e2[2 * i + 1], uint32_t(t % v.W), acc);
    } else {
      const uint64_t i = t - tasks;
      count_class(lut, h_main, h_sub, a3_pattern(v, v.e3[3 * i], v.e3[3 * i + 1], v.e3[3 * i + 2]), kPairBits3);
    }
  }
  c3_flush(acc, lut, h_g2);
  __syncthreads();
  unsigned long long* hc = hist_copy(a.hist, kExactHistStride);
  flush(h_main, hc + kMain, 256);
  flush(h_sub, hc + kSub, 256);
  flush(h_g2, hc + kG2, 256);
}

// Counting kernels keep per-class counters in LDS and flush them once per
// workgroup; a grid of a few workgroups per CU that strides over the work
// keeps those flushes (global atomics on a few hundred addresses) rare.
constexpr unsigned kCountGrid = 512;

// Workgroups of a fused counting launch: no more than are resident at once
// (with `lds` bytes of dynamic LDS each), and no more than the items need.
unsigned fused_grid(const void* kernel, size_t lds, uint64_t items, uint64_t per_block, int threads = kThreads) {
  struct Key {
    const void* kernel;
    size_t lds;
    int dev;
    bool operator<(const Key& o) const {
      return std::tie(kernel, lds, dev) < std::tie(o.kernel, o.lds, o.dev);
    }
  };
  static std::mutex mu;
  static std::map<Key, uint64_t> resident_of;
  int dev = 0;
  (void)hipGetDevice(&dev);
  uint64_t resident = 0;
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = resident_of.find(Key{kernel, lds, dev});
    if (it != resident_of.end()) resident = it->second;
  }
  if (!resident) {
    int cus = 256, per_cu = 1;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess || per_cu < 1)
      per_cu = 1;
    resident = uint64_t(cus > 0 ? cus : 256) * uint64_t(per_cu);
    std::lock_guard<std::mutex> lock(mu);
    resident_of[Key{kernel, lds, dev}] = resident;
  }
  return unsigned(std::max<uint64_t>(1, std::min<uint64_t>(resident, (items + per_block - 1) / per_block)));
}
unsigned grid_threads(uint64_t items, unsigned cap = kCountGrid, unsigned per_block = kThreads) {
  uint64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return unsigned(g);
}

}  // namespace

// Shape classes for the combine kernels (on: the identity route counted case (c)).
IdShapes id_shapes(bool on) {
  const ClassTables& t = class_tables();
  IdShapes sh;
  sh.on = on ? 1 : 0;
  // representative pair patterns (local nodes 0..3; bits: 01=0, 02=1, 12=2, 03=4, 13=5, 23=7)
  sh.path = t.lut4[(1u << 0) | (1u << 2) | (1u << 7)];
  sh.star = t.lut4[(1u << 0) | (1u << 1) | (1u << 4)];
  sh.cycle = t.lut4[(1u << 0) | (1u << 2) | (1u << 7) | (1u << 4)];
  sh.paw = t.lut4[(1u << 0) | (1u << 1) | (1u << 2) | (1u << 4)];
  sh.diamond = t.lut4[(1u << 0) | (1u << 1) | (1u << 2) | (1u << 4) | (1u << 5)];
  sh.clique = t.lut4[kPairBits4];
  return sh;
}

namespace {

// The fused counting launch of a graph with adjacency bit rows, adding to the
// kHistCopies counter copies at hist (main, sub and G2 regions, or the
// identity sums).  Returns whether the identity route ran (order 4).
bool launch_bits_count(const hm_graph* H, int k, const uint8_t* lut, unsigned long long* hist, hipStream_t st) {
  const View v = view_of(H);
  const uint64_t n2 = H->n_by_size[2], n3 = H->n_by_size[3], n4 = H->n_by_size[4];
  ExactArgs a{};
  a.v = v;
  a.n2 = n2;
  a.n3 = n3;
  a.n4 = k == 4 ? n4 : 0;
  a.lut = lut;
  a.hist = hist;
  if (k == 4) {
    const size_t rows = (size_t(v.N) * v.W + 3 * (size_t(v.N) + 1)) * 4;
    const bool lb = rows <= kLdsBitsMaxBytes;
    const bool id = use_identities(v.N, v.W);
    const size_t lds = size_t(kExact4Waves) * b4_set_words(v.W) * 4 + (lb ? rows : 0);
    const uint64_t items = n2 + (id ? v.N : 0) + n3 + (n4 + kA4Chunk - 1) / kA4Chunk;
    const void* kern = lb ? (id ? reinterpret_cast<const void*>(k_exact4_bits<true, true>)
                                : reinterpret_cast<const void*>(k_exact4_bits<true, false>))
                          : (id ? reinterpret_cast<const void*>(k_exact4_bits<false, true>)
                                : reinterpret_cast<const void*>(k_exact4_bits<false, false>));
    const unsigned grid = fused_grid(kern, lds, items, kExact4Waves, kExact4Threads);
    ProfileScope ps("k_exact4_bits", st);
    if (lb && id)
      k_exact4_bits<true, true><<<grid, kExact4Threads, lds, st>>>(a);
    else if (lb)
      k_exact4_bits<true, false><<<grid, kExact4Threads, lds, st>>>(a);
    else if (id)
      k_exact4_bits<false, true><<<grid, kExact4Threads, lds, st>>>(a);
    else
      k_exact4_bits<false, false><<<grid, kExact4Threads, lds, st>>>(a);
    return id;
  }
  const unsigned grid = fused_grid(reinterpret_cast<const void*>(k_exact3_bits), 0, n2 * v.W + n3, kThreads);
  ProfileScope ps("k_exact3_bits", st);
  k_exact3_bits<<<grid, kThreads, 0, st>>>(a);
  return false;
}

ClassMask pairs_only_mask(int k) {
  const ClassTables& t = class_tables();
  ClassMask m{{0, 0, 0, 0}};
  for (int c = 0; c < t.n_classes[k]; ++c)
    if (t.maxcard[k][c] == 2) m.w[c >> 6] |= 1ull << (c & 63);
  return m;
}

// ------------------------------------------------------- allocation-free count
// count_exact_noalloc keeps its counters and class tables in this file-scope
// device array: kHistCopies x kExactHistStride counters, then the order-4 and
// order-3 pattern->class tables.  Each device holds its own copy for the
// life of the process; host code reaches it only through the address
// hipGetSymbolAddress gives on that device.
constexpr size_t kNoAllocHistWords = size_t(kHistCopies) * kExactHistStride;
constexpr size_t kNoAllocLutBytes = 2048 + 16;
constexpr size_t kNoAllocWords = kNoAllocHistWords + (kNoAllocLutBytes + 7) / 8;
__device__ __align__(256) unsigned long long scratch[kNoAllocWords];

struct LutArg {
  uint8_t b[kNoAllocLutBytes];
};

// Clear the counter copies and write both class tables (passed by value, so
// that no host copy or device buffer is needed).
__global__ void k_noalloc_prepare(unsigned long long* __restrict__ s, LutArg luts) {
  const uint64_t i0 = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  for (uint64_t i = i0; i < kNoAllocHistWords; i += uint64_t(gridDim.x) * blockDim.x) s[i] = 0;
  uint8_t* lut = reinterpret_cast<uint8_t*>(s + kNoAllocHistWords);
  for (uint64_t i = i0; i < kNoAllocLutBytes; i += uint64_t(gridDim.x) * blockDim.x) lut[i] = luts.b[i];
}

std::mutex g_noalloc_mu;
std::vector<unsigned long long*> g_noalloc_ptr;   // per device

// The device address of `scratch` on device dev, looked up once per device.
int noalloc_scratch(int dev, unsigned long long** out) {
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (size_t(dev) >= g_noalloc_ptr.size()) g_noalloc_ptr.resize(size_t(dev) + 1, nullptr);
  if (!g_noalloc_ptr[size_t(dev)]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      set_error("hipGetSymbolAddress of the counting scratch failed on device %d: %s", dev, hipGetErrorString(e));
      return HM_EDEVICE;
    }
    g_noalloc_ptr[size_t(dev)] = static_cast<unsigned long long*>(p);
  }
  *out = g_noalloc_ptr[size_t(dev)];
  return HM_OK;
}

}  // namespace

int count_exact_impl(const hm_graph* H, int k, int64_t* counts, hipStream_t st) {
  note_use(H, st);
  const uint8_t *lut4 = nullptr, *lut3 = nullptr;
  HM_TRY(device_luts(H->device, &lut4, &lut3));
  const ClassTables& t = class_tables();
  const ClassMask pairs_only = pairs_only_mask(k);
  // H->hist is zero between calls; a call that fails part-way clears it on
  // the next call
  if (H->hist_dirty) {
    HM_TRY(fill_u64(H->hist, 0, uint64_t(kHistCopies) * kExactHistStride, st));
    H->hist_dirty = false;
  }
  struct DirtyOnError {
    const hm_graph* H;
    bool ok = false;
    ~DirtyOnError() {
      if (!ok) H->hist_dirty = true;
    }
  } guard{H};
  const uint64_t n3 = H->n_by_size[3], n4 = H->n_by_size[4];
  const View v = view_of(H);
  bool id = false;
  if (v.bits) {
    id = launch_bits_count(H, k, k == 4 ? lut4 : lut3, H->hist, st);
  } else {
    if (k == 4 && n4) {
      ProfileScope ps("k_case_a4", st);
      k_case_a4<<<grid_threads(n4), kThreads, 0, st>>>(v, n4, lut4, H->hist);
    }
    if (k == 3 && n3) {
      ProfileScope ps("k_case_a3", st);
      k_case_a3<<<grid_threads(n3), kThreads, 0, st>>>(v, n3, lut3, H->hist);
    }
    HM_HIP(hipGetLastError());
    HM_TRY(count_sparse(H, k, st));
  }
  HM_HIP(hipGetLastError());
  k_combine<<<1, 256, 0, st>>>(H->hist, t.n_classes[k], pairs_only, counts, id_shapes(id));
  HM_HIP(hipGetLastError());
  guard.ok = true;
  return HM_OK;
}

}  // namespace hm

extern "C" int count_exact(const hm_graph* H, int k, int64_t* counts, void* stream) {
  try {
    if (!H || !counts) {
      hm::set_error("NULL argument to count_exact");
      return HM_EINVAL;
    }
    if (k != 3 && k != 4) {
      hm::set_error("order %d is not supported (3 or 4)", k);
      return HM_EUNSUPPORTED;
    }
    return hm::count_exact_impl(H, k, counts, static_cast<hipStream_t>(stream));
  } catch (...) {
    return hm::api_failure();
  }
}

extern "C" int count_exact_noalloc(const hm_graph* H, int k, int64_t* counts, void* stream) {
  try {
    if (!H || !counts) {
      hm::set_error("NULL argument to count_exact_noalloc");
      return HM_EINVAL;
    }
    if (k != 3 && k != 4) {
      hm::set_error("order %d is not supported (3 or 4)", k);
      return HM_EUNSUPPORTED;
    }
    if (!H->bits) {
      hm::set_error("count_exact_noalloc counts graphs with adjacency bit rows only (at most %u nodes); this one has "
                    "%u, and counting it without bit rows needs temporaries sized by the graph",
                    hm::bitset_max_nodes(), H->n_nodes);
      return HM_EUNSUPPORTED;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != H->device) {
      (void)hipGetLastError();
      hm::set_error("count_exact_noalloc: the graph lives on device %d, the current device is %d", H->device, dev);
      return HM_EINVAL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned long long* s = nullptr;
    HM_TRY(hm::noalloc_scratch(dev, &s));
    hm::note_use(H, st);
    const hm::ClassTables& t = hm::class_tables();
    hm::LutArg luts;
    std::memcpy(luts.b, t.lut4, 2048);
    std::memcpy(luts.b + 2048, t.lut3, 16);
    hm::k_noalloc_prepare<<<16, 256, 0, st>>>(s, luts);
    HM_HIP(hipGetLastError());
    const uint8_t* lut = reinterpret_cast<const uint8_t*>(s + hm::kNoAllocHistWords) + (k == 4 ? 0 : 2048);
    const bool id = hm::launch_bits_count(H, k, lut, s, st);
    HM_HIP(hipGetLastError());
    hm::k_combine<<<1, 256, 0, st>>>(s, t.n_classes[k], hm::pairs_only_mask(k), counts, hm::id_shapes(id));
    HM_HIP(hipGetLastError());
    return HM_OK;
  } catch (...) {
    return hm::api_failure();
  }
}
